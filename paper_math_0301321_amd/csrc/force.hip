// Material force, sub-step 1 of the time step (Sec. 3.2), in FP64.
//
// One thread per marker gathers every term that acts on it (lattice stretch
// edges, bend triples in which it is an end or the centre, springs through a
// CSR adjacency, its tether), so no two threads write the same output and the
// result does not depend on scheduling.  Each edge / triple is evaluated once
// per marker it touches; the window drive is added through a per-marker slot
// of the drive list.  Lattice rest lengths and bend scales come from the
// reference shape and weights, computed once when those are set.  In the time
// step the same pass also writes the marker's sorted record for the spreading.  Force laws: see include/ib.h.
// With displacements as the state (DISP: X holds D = X - Y, Y = X_ref) an
// edge vector is (Yo - Yq) + (Do - Dq), a second difference Da - 2Dc + Db and
// a tether offset D itself, each with the relative precision of D.
#include "dev_common.h"
#include "ib_internal.h"

namespace ib {

struct V3 {
  double x, y, z;
};

__device__ __forceinline__ V3 ld3(const double *__restrict__ A, int64_t M, int64_t q) {
  return V3{A[q], A[M + q], A[2 * M + q]};
}
// Length and second difference with their roundings fixed by explicit fused
// multiply-adds, so that the values formed from the reference shape when it
// is set and those formed from the positions at every step are the same
// double for equal inputs: the force vanishes exactly at the reference shape.
__device__ __forceinline__ double nrm(const V3 &a) { return sqrt(fma(a.x, a.x, fma(a.y, a.y, a.z * a.z))); }
__device__ __forceinline__ V3 second_diff(const V3 &a, const V3 &c, const V3 &b) {
  return V3{fma(-2.0, c.x, a.x) + b.x, fma(-2.0, c.y, a.y) + b.y, fma(-2.0, c.z, a.z) + b.z};
}

// Reference-shape constants of a lattice marker q = (i1, i2), [12][M]:
//   0, 1: rest length Le of the edge (q, q + 1 along index 1) and Ks w / Le^2
//         (w the mean of the two endpoint weights);
//   2, 3: the same for the edge to the next row (index 2, wrapping when periodic);
//   4, 5: Kb w_q / Lc^4 of the bend triples centred at q along index 1 and 2
//         (Lc the mean rest length of the triple's two edges);
//   6 .. 8, 9 .. 11: the reference second difference Y_a - 2 Y_q + Y_b of
//         those two triples (x, y, z);
// zero where the edge or triple does not exist.  They depend only on X_ref and
// w, so they are computed when those are set; the stiffness multipliers k are
// applied at run time.
__global__ __launch_bounds__(256) void k_lattice_pre(Material m, double *__restrict__ pre) {
  const int64_t q = gtid();
  const int64_t M = m.M;
  if (q >= M) return;
  double v[kLatPre] = {};
  for (int l = 0; l < m.lat.n; l++) {
    const LatticeDev &L = m.lat.l[l];
    if (q < L.first || q >= L.first + (int64_t)L.n1 * L.n2) continue;
    const int64_t rel = q - L.first, n1 = L.n1, n2 = L.n2;
    const int64_t i1 = rel % n1, i2 = rel / n1;
    const bool per = L.periodic2 != 0;
    auto idx = [&](int64_t a1, int64_t a2) { return L.first + a2 * n1 + a1; };
    auto w2 = [&](int64_t a2) { return per ? (a2 + n2) % n2 : a2; };
    const V3 yq = ld3(m.X_ref, M, q);
    auto edge = [&](int64_t o, double &le, double &ke) {
      const V3 yo = ld3(m.X_ref, M, o);
      const V3 dy{yo.x - yq.x, yo.y - yq.y, yo.z - yq.z};
      le = nrm(dy);
      ke = L.Ks * (0.5 * (m.w[q] + m.w[o])) / (le * le);
    };
    auto bend = [&](int64_t a, int64_t b, double *d2) {
      const V3 ya = ld3(m.X_ref, M, a), yb = ld3(m.X_ref, M, b);
      const V3 e1{yq.x - ya.x, yq.y - ya.y, yq.z - ya.z}, e2{yb.x - yq.x, yb.y - yq.y, yb.z - yq.z};
      const double Lc = 0.5 * (nrm(e1) + nrm(e2));
      const V3 dy = second_diff(ya, yq, yb);
      d2[0] = dy.x;
      d2[1] = dy.y;
      d2[2] = dy.z;
      return L.Kb * m.w[q] / (Lc * Lc * Lc * Lc);
    };
    if (L.Ks != 0.0) {
      if (i1 < n1 - 1) edge(idx(i1 + 1, i2), v[0], v[1]);
      if (per || i2 < n2 - 1) edge(idx(i1, w2(i2 + 1)), v[2], v[3]);
    }
    if (L.Kb != 0.0) {
      if (i1 >= 1 && i1 <= n1 - 2) v[4] = bend(idx(i1 - 1, i2), idx(i1 + 1, i2), v + 6);
      if (per || (i2 >= 1 && i2 <= n2 - 2)) v[5] = bend(idx(i1, w2(i2 - 1)), idx(i1, w2(i2 + 1)), v + 9);
    }
    break;
  }
  for (int j = 0; j < kLatPre; j++) pre[j * M + q] = v[j];
}

// Edge vector from q to o: Xo - Xq, or with displacements (Yo - Yq) + (Do - Dq).
template <bool DISP>
__device__ __forceinline__ V3 edge_vec(const V3 &xq, const V3 &xo, const V3 &yq, const V3 &yo) {
  if (DISP) return V3{(yo.x - yq.x) + (xo.x - xq.x), (yo.y - yq.y) + (xo.y - xq.y), (yo.z - yq.z) + (xo.z - xq.z)};
  return V3{xo.x - xq.x, xo.y - xq.y, xo.z - xq.z};
}

// Force on marker q (state xq, reference yq, multiplier kq) from the stretch
// edge to o (xo, yo, ko) with rest length le and ke = Ks w / le^2 (of the
// edge's lower endpoint); the reference positions are read only with DISP.
// Extension |d| - le of a lattice edge; with displacements (d = dy + dl,
// dy = Yo - Yq, dl = Do - Dq) formed as (2 dy.dl + dl.dl) / (|d| + le), without
// the cancellation of two lengths that agree to the strain.
template <bool DISP>
__device__ __forceinline__ double extension(const V3 &xq, const V3 &xo, const V3 &yq, const V3 &yo, double len,
                                            double le) {
  if (!DISP) return len - le;
  const V3 dy{yo.x - yq.x, yo.y - yq.y, yo.z - yq.z}, dl{xo.x - xq.x, xo.y - xq.y, xo.z - xq.z};
  const double num = 2.0 * (dy.x * dl.x + dy.y * dl.y + dy.z * dl.z) + (dl.x * dl.x + dl.y * dl.y + dl.z * dl.z);
  return num / (len + le);
}

template <bool DISP>
__device__ __forceinline__ void stretch_on(const V3 &xq, const V3 &yq, double kq, const V3 &xo, const V3 &yo,
                                           double ko, double le, double ke, V3 &f) {
  const V3 d = edge_vec<DISP>(xq, xo, yq, yo);
  const double len = nrm(d);
  const double s = ke * (0.5 * (kq + ko)) * extension<DISP>(xq, xo, yq, yo, len, le) / len;
  f.x += s * d.x;
  f.y += s * d.y;
  f.z += s * d.z;
}

// Force on marker q from the bend triple with positions xa, xc (centre c,
// multiplier kc), xb, cb = Kb w_c / Lc^4 and d2 (3 strided values) the
// reference second difference Y_a - 2 Y_c + Y_b; role: 0 = end, 1 = centre.
template <bool DISP>
__device__ __forceinline__ void bend_on(const Material &m, const V3 &xa, const V3 &xc, const V3 &xb, int64_t c,
                                        double kc, int role, double cb, const double *__restrict__ d2, V3 &f) {
  const int64_t M = m.M;
  const V3 dx = second_diff(xa, xc, xb);
  V3 v = dx;                                   // with displacements: Da - 2Dc + Db
  if (!DISP) {
    const V3 y2 = ld3(d2, M, c);
    v = V3{dx.x - y2.x, dx.y - y2.y, dx.z - y2.z};
  }
  const double K = cb * kc;
  const double s = role ? 2.0 * K : -K;
  f.x += s * v.x;
  f.y += s * v.y;
  f.z += s * v.z;
}

template <bool DISP>
__device__ void lattice_force(const Material &m, const LatticeDev &L, const double *__restrict__ X,
                              int64_t q, const V3 &xq, V3 &f) {
  const int64_t M = m.M;
  const double *P = m.lat_pre;
  const int64_t rel = q - L.first;
  const int64_t n1 = L.n1, n2 = L.n2;
  const int64_t i1 = rel % n1, i2 = rel / n1;
  const bool per = L.periodic2 != 0;
  auto idx = [&](int64_t a1, int64_t a2) { return L.first + a2 * n1 + a1; };
  auto w2 = [&](int64_t a2) { return per ? (a2 + n2) % n2 : a2; };
  const bool has_dn = per || i2 > 0, has_up = per || i2 < n2 - 1;
  if (L.Ks == 0.0 && L.Kb == 0.0) return;
  // the four neighbours' positions and multipliers, read once for the edges and the bends
  const int64_t q1m = idx(i1 - 1, i2), q1p = idx(i1 + 1, i2), q2m = idx(i1, w2(i2 - 1)), q2p = idx(i1, w2(i2 + 1));
  V3 x1m{}, x1p{}, x2m{}, x2p{};
  double k1m = 0.0, k1p = 0.0, k2m = 0.0, k2p = 0.0;
  if (i1 > 0) { x1m = ld3(X, M, q1m); k1m = m.k[q1m]; }
  if (i1 < n1 - 1) { x1p = ld3(X, M, q1p); k1p = m.k[q1p]; }
  if (has_dn) { x2m = ld3(X, M, q2m); k2m = m.k[q2m]; }
  if (has_up) { x2p = ld3(X, M, q2p); k2p = m.k[q2p]; }
  const double kq = m.k[q];
  if (L.Ks != 0.0) {
    // reference positions of q and the four neighbours (edge vectors with displacements)
    V3 yq{}, y1m{}, y1p{}, y2m{}, y2p{};
    if (DISP) {
      yq = ld3(m.X_ref, M, q);
      if (i1 > 0) y1m = ld3(m.X_ref, M, q1m);
      if (i1 < n1 - 1) y1p = ld3(m.X_ref, M, q1p);
      if (has_dn) y2m = ld3(m.X_ref, M, q2m);
      if (has_up) y2p = ld3(m.X_ref, M, q2p);
    }
    if (i1 > 0) stretch_on<DISP>(xq, yq, kq, x1m, y1m, k1m, P[q1m], P[M + q1m], f);
    if (i1 < n1 - 1) stretch_on<DISP>(xq, yq, kq, x1p, y1p, k1p, P[q], P[M + q], f);
    if (has_dn) stretch_on<DISP>(xq, yq, kq, x2m, y2m, k2m, P[2 * M + q2m], P[3 * M + q2m], f);
    if (has_up) stretch_on<DISP>(xq, yq, kq, x2p, y2p, k2p, P[2 * M + q], P[3 * M + q], f);
  }
  if (L.Kb != 0.0) {
    const double *C1 = P + 4 * M, *C2 = P + 5 * M, *D1 = P + 6 * M, *D2 = P + 9 * M;
    // Along each direction the triples containing q are centred at q, at its
    // successor and at its predecessor (in that order); they need the
    // positions at offsets -2 .. 2, each read once.
    // direction 1: centres 1 .. n1-2 (the neighbours exist wherever a triple does)
    {
      const bool b0 = i1 >= 1 && i1 <= n1 - 2, bp = i1 + 1 <= n1 - 2, bm = i1 - 1 >= 1;
      V3 xm2{}, xp2{};
      if (bm) xm2 = ld3(X, M, idx(i1 - 2, i2));
      if (bp) xp2 = ld3(X, M, idx(i1 + 2, i2));
      if (b0) bend_on<DISP>(m, x1m, xq, x1p, q, kq, 1, C1[q], D1, f);
      if (bp) bend_on<DISP>(m, xq, x1p, xp2, q1p, k1p, 0, C1[q1p], D1, f);
      if (bm) bend_on<DISP>(m, xm2, x1m, xq, q1m, k1m, 0, C1[q1m], D1, f);
    }
    // direction 2: centres 1 .. n2-2, or every row when periodic
    {
      auto centre_ok = [&](int64_t c2) { return per || (c2 >= 1 && c2 <= n2 - 2); };
      const bool b0 = centre_ok(i2), bp = (per || i2 + 1 < n2) && centre_ok(i2 + 1),
                 bm = (per || i2 - 1 >= 0) && centre_ok(i2 - 1);
      V3 xm2{}, xp2{};
      if (bm) xm2 = ld3(X, M, idx(i1, w2(i2 - 2)));
      if (bp) xp2 = ld3(X, M, idx(i1, w2(i2 + 2)));
      if (b0) bend_on<DISP>(m, x2m, xq, x2p, q, kq, 1, C2[q], D2, f);
      if (bp) bend_on<DISP>(m, xq, x2p, xp2, q2p, k2p, 0, C2[q2p], D2, f);
      if (bm) bend_on<DISP>(m, xm2, x2m, xq, q2m, k2m, 0, C2[q2m], D2, f);
    }
  }
}

// Elastic force on marker q (every term except the drive).
template <bool DISP>
__device__ __forceinline__ V3 marker_force(const Material &m, const double *__restrict__ X, int64_t q,
                                           const V3 &xq) {
  const int64_t M = m.M;
  V3 f{0.0, 0.0, 0.0};
  for (int l = 0; l < m.lat.n; l++) {
    const LatticeDev &L = m.lat.l[l];
    if (q >= L.first && q < L.first + (int64_t)L.n1 * L.n2) {
      lattice_force<DISP>(m, L, X, q, xq, f);
      break;
    }
  }
  if (m.sp_rowptr) {
    const V3 yq = DISP ? ld3(m.X_ref, M, q) : V3{};
    for (int32_t e = m.sp_rowptr[q]; e < m.sp_rowptr[q + 1]; e++) {
      const int64_t o = m.sp_col[e];
      const V3 xo = ld3(X, M, o);
      const V3 d = edge_vec<DISP>(xq, xo, yq, DISP ? ld3(m.X_ref, M, o) : V3{});
      const double len = nrm(d);
      const double K = m.K_spring * (0.5 * (m.k[q] + m.k[o]));
      const double s = K * (len - m.sp_rest[e]) / len;
      f.x += s * d.x;
      f.y += s * d.y;
      f.z += s * d.z;
    }
  }
  if (m.kappa) {
    const double kw = m.kappa[q] * m.w[q];
    if (kw != 0.0) {
      if (DISP) {            // the offset from the reference is the displacement
        f.x += -kw * xq.x;
        f.y += -kw * xq.y;
        f.z += -kw * xq.z;
      } else {
        const V3 y = ld3(m.X_ref, M, q);
        f.x += -kw * (xq.x - y.x);
        f.y += -kw * (xq.y - y.y);
        f.z += -kw * (xq.z - y.z);
      }
    }
  }
  return f;
}

// Window drive (Sec. 4) on marker q: amp = A sin(2 pi f t) evaluated on the
// host in FP64, times w_q, along the marker's direction (slot j of the drive list).
__device__ __forceinline__ void add_drive(const Material &m, const int32_t *__restrict__ slot,
                                          const double *__restrict__ dir, int64_t D, double amp, int64_t q, V3 &f) {
  if (!slot || amp == 0.0) return;
  const int j = slot[q];
  if (j < 0) return;
  const double s = amp * m.w[q];
  f.x += s * dir[j];
  f.y += s * dir[D + j];
  f.z += s * dir[2 * D + j];
}

template <bool DISP>
__global__ __launch_bounds__(256) void k_force(Material m, const double *__restrict__ X,
                                               const int32_t *__restrict__ slot, const double *__restrict__ dir,
                                               int64_t D, double amp, double *__restrict__ F) {
  const int64_t q = (int64_t)xcd_runs<16>(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;   // lattice neighbours on one L2
  const int64_t M = m.M;
  if (q >= M) return;
  const V3 xq = ld3(X, M, q);
  V3 f = marker_force<DISP>(m, X, q, xq);
  add_drive(m, slot, dir, D, amp, q, f);
  F[q] = f.x;
  F[M + q] = f.y;
  F[2 * M + q] = f.z;
}

// Force and sorted record in one pass: the record of marker q (fractional
// offsets and cell key from X as the binning forms them, force in the fluid
// precision) goes to its sorted position inv[q]; the FP64 force is written
// only when asked for.
template <typename T, bool DISP>
__global__ __launch_bounds__(256) void k_force_rec(Material m, const double *__restrict__ X,
                                                   const int32_t *__restrict__ slot, const double *__restrict__ dir,
                                                   int64_t D, double amp, const int32_t *__restrict__ inv, double h,
                                                   int n, int nz, int log2nt, double *__restrict__ F,
                                                   Rec<T> *__restrict__ recs) {
  const int64_t q = (int64_t)xcd_runs<16>(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;   // lattice neighbours on one L2
  const int64_t M = m.M;
  if (q >= M) return;
  const V3 xq = ld3(X, M, q);
  V3 f = marker_force<DISP>(m, X, q, xq);
  add_drive(m, slot, dir, D, amp, q, f);
  if (F) {
    F[q] = f.x;
    F[M + q] = f.y;
    F[2 * M + q] = f.z;
  }
  Rec<T> r{};
  V3 pq = xq;                                  // the position, where the delta function is evaluated
  if (DISP) {
    const V3 yq = ld3(m.X_ref, M, q);
    pq = V3{yq.x + xq.x, yq.y + xq.y, yq.z + xq.z};
  }
  const double xs[3] = {pq.x, pq.y, pq.z};
  int cc[3];
  for (int d = 0; d < 3; d++) {
    const double s = xs[d] / h;
    const double fl = floor(s);
    r.f[d] = (T)(s - fl);
    const int64_t ci = isfinite(s) ? (int64_t)fl : 0;
    cc[d] = d == 2 ? wrap_cell(ci, nz) : (int)(ci & (int64_t)(n - 1));   // as the binning wraps
  }
  r.F[0] = (T)f.x;
  r.F[1] = (T)f.y;
  r.F[2] = (T)f.z;
  r.key = cell_key(cc[0], cc[1], cc[2], log2nt);
  recs[inv[q]] = r;
}

hipError_t launch_lattice_pre(ib_ctx *c) {
  if (c->M == 0 || !c->ws.lat_pre) return hipSuccess;
  hipLaunchKernelGGL(k_lattice_pre, dim3((unsigned)((c->M + 255) / 256)), dim3(256), 0, c->stream, c->mat,
                     c->ws.lat_pre);
  return hipGetLastError();
}

hipError_t launch_force(ib_ctx *c, const double *X, double amp, double *F) {
  if (c->M == 0) return hipSuccess;
  PhaseScope ps(c, PH_FORCE);
  if (c->mat.disp)
    hipLaunchKernelGGL(k_force<true>, dim3((unsigned)((c->M + 255) / 256)), dim3(256), 0, c->stream, c->mat, X,
                       c->ws.drive_slot, c->ws.drive_dir, c->n_drive, amp, F);
  else
    hipLaunchKernelGGL(k_force<false>, dim3((unsigned)((c->M + 255) / 256)), dim3(256), 0, c->stream, c->mat, X,
                       c->ws.drive_slot, c->ws.drive_dir, c->n_drive, amp, F);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_force_rec(ib_ctx *c, const double *X, double amp, double *F) {
  if (c->M == 0) return hipSuccess;
  PhaseScope ps(c, PH_FORCE);
  hipLaunchKernelGGL((c->mat.disp ? k_force_rec<T, true> : k_force_rec<T, false>),
                     dim3((unsigned)((c->M + 255) / 256)), dim3(256), 0, c->stream, c->mat, X,
                     c->ws.drive_slot, c->ws.drive_dir, c->n_drive, amp, c->ws.inv, c->h, c->n, c->nz, c->log2nt, F,
                     (Rec<T> *)c->ws.recs);
  return hipGetLastError();
}

template hipError_t launch_force_rec<float>(ib_ctx *, const double *, double, double *);
template hipError_t launch_force_rec<double>(ib_ctx *, const double *, double, double *);

// launch_force_rec passes amp as argument kForceRecAmpArg of k_force_rec
template <typename T>
const void *force_rec_kernel(bool disp) {
  return disp ? reinterpret_cast<const void *>(&k_force_rec<T, true>)
              : reinterpret_cast<const void *>(&k_force_rec<T, false>);
}
template const void *force_rec_kernel<float>(bool);
template const void *force_rec_kernel<double>(bool);

}  // namespace ib

// ---------------------------------------------------------------------------
// Adjoint of the force: with fbar the force cotangent,
//   Xbar_q -= (H fbar)_q   (H the Hessian of the elastic energy; f = -grad E),
//   kbar_q += (df/dk_q) . fbar   (f is linear in k).
// Gather form, one thread per marker, as in the forward kernel.
// ---------------------------------------------------------------------------
namespace ib {

// Stretch or spring edge (q, o) with energy 1/2 Ku kf (|d| - L0)^2 / D, D = L0^2
// (lattice) or 1 (spring), d = Xo - Xq.  Adds the edge's part of (H fbar)_q to hv
// and returns (unit-kf edge force) . fbar over both endpoints.
__device__ __forceinline__ double edge_adj(const Material &m, const double *__restrict__ X,
                                           const double *__restrict__ fb, int64_t M, int64_t q, int64_t o, double Ku,
                                           double kf, double L0, bool rest_sq, V3 &hv) {
  const V3 xq = ld3(X, M, q), xo = ld3(X, M, o);
  const V3 vq = ld3(fb, M, q), vo = ld3(fb, M, o);
  V3 yq{}, yo{};
  if (m.disp) {
    yq = ld3(m.X_ref, M, q);
    yo = ld3(m.X_ref, M, o);
  }
  const V3 d = m.disp ? edge_vec<true>(xq, xo, yq, yo) : edge_vec<false>(xq, xo, yq, yo);
  const V3 dv{vo.x - vq.x, vo.y - vq.y, vo.z - vq.z};
  const double len = nrm(d);
  // |d| - L0; a lattice edge (rest_sq: L0 = |Yo - Yq|) from displacements as in the force
  const double ext = (rest_sq && m.disp) ? extension<true>(xq, xo, yq, yo, len, L0) : len - L0;
  const double Kup = rest_sq ? Ku / (L0 * L0) : Ku;
  const double Kp = Kup * kf;
  const double dd = d.x * dv.x + d.y * dv.y + d.z * dv.z;
  const double a = ext / len, b = (L0 / (len * len * len)) * dd;
  hv.x -= Kp * (a * dv.x + b * d.x);
  hv.y -= Kp * (a * dv.y + b * d.y);
  hv.z -= Kp * (a * dv.z + b * d.z);
  return -(Kup * ext / len) * dd;
}

// The lattice part of (H fbar)_q and of kbar_q, as the forward kernel forms
// the force: the neighbours' states, cotangents and multipliers read once
// (offsets -2 .. 2 along each direction), the rest lengths, stiffness
// scales and reference second differences from the lattice constants.
template <bool DISP>
__device__ void lattice_hessvec(const Material &m, const LatticeDev &L, const double *__restrict__ X,
                                const double *__restrict__ fb, int64_t q, V3 &hv, double &kb) {
  const int64_t M = m.M;
  const double *P = m.lat_pre;
  const int64_t rel = q - L.first;
  const int64_t n1 = L.n1, n2 = L.n2;
  const int64_t i1 = rel % n1, i2 = rel / n1;
  const bool per = L.periodic2 != 0;
  auto idx = [&](int64_t a1, int64_t a2) { return L.first + a2 * n1 + a1; };
  auto w2 = [&](int64_t a2) { return per ? (a2 + n2) % n2 : a2; };
  const bool has_dn = per || i2 > 0, has_up = per || i2 < n2 - 1;
  if (L.Ks == 0.0 && L.Kb == 0.0) return;
  const int64_t q1m = idx(i1 - 1, i2), q1p = idx(i1 + 1, i2), q2m = idx(i1, w2(i2 - 1)), q2p = idx(i1, w2(i2 + 1));
  const V3 xq = ld3(X, M, q), vq = ld3(fb, M, q);
  const double kq = m.k[q];
  V3 x1m{}, x1p{}, x2m{}, x2p{}, v1m{}, v1p{}, v2m{}, v2p{};
  double k1m = 0.0, k1p = 0.0, k2m = 0.0, k2p = 0.0;
  if (i1 > 0) { x1m = ld3(X, M, q1m); v1m = ld3(fb, M, q1m); k1m = m.k[q1m]; }
  if (i1 < n1 - 1) { x1p = ld3(X, M, q1p); v1p = ld3(fb, M, q1p); k1p = m.k[q1p]; }
  if (has_dn) { x2m = ld3(X, M, q2m); v2m = ld3(fb, M, q2m); k2m = m.k[q2m]; }
  if (has_up) { x2p = ld3(X, M, q2p); v2p = ld3(fb, M, q2p); k2p = m.k[q2p]; }
  if (L.Ks != 0.0) {
    V3 yq{}, y1m{}, y1p{}, y2m{}, y2p{};
    if (DISP) {
      yq = ld3(m.X_ref, M, q);
      if (i1 > 0) y1m = ld3(m.X_ref, M, q1m);
      if (i1 < n1 - 1) y1p = ld3(m.X_ref, M, q1p);
      if (has_dn) y2m = ld3(m.X_ref, M, q2m);
      if (has_up) y2p = ld3(m.X_ref, M, q2p);
    }
    // edge (q, o): energy 1/2 ke kf (|d| - le)^2, ke = Ks w / le^2, kf the mean multiplier
    auto edge = [&](const V3 &xo, const V3 &yo, const V3 &vo, double ko, double le, double ke) {
      const V3 d = edge_vec<DISP>(xq, xo, yq, yo);
      const V3 dv{vo.x - vq.x, vo.y - vq.y, vo.z - vq.z};
      const double len = nrm(d);
      const double ext = extension<DISP>(xq, xo, yq, yo, len, le);
      const double Kp = ke * (0.5 * (kq + ko));
      const double dd = d.x * dv.x + d.y * dv.y + d.z * dv.z;
      const double a = ext / len, b = (le / (len * len * len)) * dd;
      hv.x -= Kp * (a * dv.x + b * d.x);
      hv.y -= Kp * (a * dv.y + b * d.y);
      hv.z -= Kp * (a * dv.z + b * d.z);
      kb += 0.5 * (-(ke * ext / len) * dd);
    };
    if (i1 > 0) edge(x1m, y1m, v1m, k1m, P[q1m], P[M + q1m]);
    if (i1 < n1 - 1) edge(x1p, y1p, v1p, k1p, P[q], P[M + q]);
    if (has_dn) edge(x2m, y2m, v2m, k2m, P[2 * M + q2m], P[3 * M + q2m]);
    if (has_up) edge(x2p, y2p, v2p, k2p, P[2 * M + q], P[3 * M + q]);
  }
  if (L.Kb != 0.0) {
    const double *C1 = P + 4 * M, *C2 = P + 5 * M, *D1 = P + 6 * M, *D2 = P + 9 * M;
    // triple (a, c, b): z = fbar_a - 2 fbar_c + fbar_b; K = cb k_c with cb = Kb w_c / Lc^4;
    // q at an end adds K z, q the centre adds -2 K z and kbar_q gets -cb (v . z),
    // v the second difference of the state less the reference one
    auto zdiff = [](const V3 &a, const V3 &c, const V3 &b) {
      return V3{a.x - 2.0 * c.x + b.x, a.y - 2.0 * c.y + b.y, a.z - 2.0 * c.z + b.z};
    };
    auto end = [&](const V3 &z, double cb, double kc) {
      const double K = cb * kc;
      hv.x += K * z.x;
      hv.y += K * z.y;
      hv.z += K * z.z;
    };
    auto centre = [&](const V3 &z, double cb, const V3 &xa, const V3 &xb, const double *d2) {
      const double K = cb * kq;
      hv.x += -2.0 * K * z.x;
      hv.y += -2.0 * K * z.y;
      hv.z += -2.0 * K * z.z;
      const V3 dx = second_diff(xa, xq, xb);
      V3 v = dx;                                   // with displacements: Da - 2Dq + Db
      if (!DISP) {
        const V3 y2 = ld3(d2, M, q);
        v = V3{dx.x - y2.x, dx.y - y2.y, dx.z - y2.z};
      }
      kb += -cb * (v.x * z.x + v.y * z.y + v.z * z.z);
    };
    // direction 1: centres 1 .. n1-2
    {
      const bool b0 = i1 >= 1 && i1 <= n1 - 2, bp = i1 + 1 <= n1 - 2, bm = i1 - 1 >= 1;
      V3 vm2{}, vp2{};
      if (bm) vm2 = ld3(fb, M, idx(i1 - 2, i2));
      if (bp) vp2 = ld3(fb, M, idx(i1 + 2, i2));
      if (b0) centre(zdiff(v1m, vq, v1p), C1[q], x1m, x1p, D1);
      if (bp) end(zdiff(vq, v1p, vp2), C1[q1p], k1p);
      if (bm) end(zdiff(vm2, v1m, vq), C1[q1m], k1m);
    }
    // direction 2: centres 1 .. n2-2, or every row when periodic
    {
      auto centre_ok = [&](int64_t c2) { return per || (c2 >= 1 && c2 <= n2 - 2); };
      const bool b0 = centre_ok(i2), bp = (per || i2 + 1 < n2) && centre_ok(i2 + 1),
                 bm = (per || i2 - 1 >= 0) && centre_ok(i2 - 1);
      V3 vm2{}, vp2{};
      if (bm) vm2 = ld3(fb, M, idx(i1, w2(i2 - 2)));
      if (bp) vp2 = ld3(fb, M, idx(i1, w2(i2 + 2)));
      if (b0) centre(zdiff(v2m, vq, v2p), C2[q], x2m, x2p, D2);
      if (bp) end(zdiff(vq, v2p, vp2), C2[q2p], k2p);
      if (bm) end(zdiff(vm2, v2m, vq), C2[q2m], k2m);
    }
  }
}

template <bool DISP>
__global__ __launch_bounds__(256) void k_hessvec(Material m, const double *__restrict__ X,
                                                 const double *__restrict__ fb, double *__restrict__ Xbar,
                                                 double *__restrict__ kbar) {
  const int64_t q = gtid();
  const int64_t M = m.M;
  if (q >= M) return;
  // the values indexed by q alone, loaded together before the terms that use
  // them (the tether sits behind branches; the outputs are read-modify-write)
  const double kw = m.kappa ? m.kappa[q] * m.w[q] : 0.0;
  const V3 fq = ld3(fb, M, q);
  const double xb0 = Xbar[q], xb1 = Xbar[M + q], xb2 = Xbar[2 * M + q], kb0 = kbar[q];
  V3 hv{0.0, 0.0, 0.0};
  double kb = 0.0;
  for (int l = 0; l < m.lat.n; l++) {
    const LatticeDev &L = m.lat.l[l];
    if (q >= L.first && q < L.first + (int64_t)L.n1 * L.n2) {
      lattice_hessvec<DISP>(m, L, X, fb, q, hv, kb);
      break;
    }
  }
  if (m.sp_rowptr) {
    for (int32_t e = m.sp_rowptr[q]; e < m.sp_rowptr[q + 1]; e++) {
      const int64_t o = m.sp_col[e];
      const double kf = 0.5 * (m.k[q] + m.k[o]);
      kb += 0.5 * edge_adj(m, X, fb, M, q, o, m.K_spring, kf, m.sp_rest[e], false, hv);
    }
  }
  if (kw != 0.0) {
    hv.x += kw * fq.x;
    hv.y += kw * fq.y;
    hv.z += kw * fq.z;
  }
  Xbar[q] = xb0 - hv.x;
  Xbar[M + q] = xb1 - hv.y;
  Xbar[2 * M + q] = xb2 - hv.z;
  kbar[q] = kb0 + kb;
}

hipError_t launch_hessvec(ib_ctx *c, const double *X, const double *v, double *Xbar, double *kbar) {
  if (c->M == 0) return hipSuccess;
  PhaseScope ps(c, PH_HESSVEC);
  hipLaunchKernelGGL((c->mat.disp ? k_hessvec<true> : k_hessvec<false>), dim3((unsigned)((c->M + 255) / 256)),
                     dim3(256), 0, c->stream, c->mat, X, v, Xbar, kbar);
  return hipGetLastError();
}

}  // namespace ib
