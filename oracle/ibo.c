/*
 * ibo.c -- ORACLE for the immersed-boundary time step (plain FP64, CPU).
 *
 * TEST INFRASTRUCTURE ONLY: called by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  Shares no
 * code with the GPU library.  Compiled with -O2 -ffp-contract=off, no
 * fast-math, so every operation is an IEEE FP64 round-to-nearest operation in
 * the order written.
 *
 * Every function follows one passage of Givelberg & Bunn, Sec. 3; each says
 * which.  Loops are plain: markers in index order, grid points in memory
 * order.  OpenMP is used only where iterations are independent (pencils of
 * the FFT, grid points of the advection, markers of the interpolation), so
 * the results do not depend on the thread count.
 */
#include "ibo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

int ibo_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void ibo_set_num_threads(int nt) {
#ifdef _OPENMP
  if (nt > 0) omp_set_num_threads(nt);
#else
  (void)nt;
#endif
}

static inline int64_t wrap(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

/* node (i, j, k) of the N x N x Nz grid, wrapped periodically */
static inline int64_t gidx(int64_t N, int64_t Nz, int64_t i, int64_t j, int64_t k) {
  return (wrap(k, Nz) * N + wrap(j, N)) * N + wrap(i, N);
}

/* ------------------------------------------------------------------------
 * phi, Sec. 3.2 (definition of delta_h): the piecewise formula as printed,
 * evaluated at |r|, the outer branch through the inner one.
 * ---------------------------------------------------------------------- */
double ibo_phi(double r) {
  double a = fabs(r);
  if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
  if (a <= 2.0) return 0.5 - ibo_phi(2.0 - a);
  return 0.0;
}

/* ------------------------------------------------------------------------
 * Binning (the grid/marker partition of Sec. 3.3).  The cell of a marker is
 * the node floor(X/h) in each dimension, wrapped periodically.  Cells are
 * grouped in blocks of 8 x 8 x 8; markers are ordered by block (linear block
 * index, x fastest), then by cell within the block (x fastest), ties by
 * marker id.
 * ---------------------------------------------------------------------- */
typedef struct { uint32_t key; int32_t id; } kv_t;

static int kv_cmp(const void *a, const void *b) {
  const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->id > y->id) - (x->id < y->id);
}

void ibo_bin(int N, int Nz, double L, int64_t M, const double *X, uint32_t *keys_sorted, int32_t *perm) {
  double h = L / N;
  kv_t *kv = (kv_t *)malloc(sizeof(kv_t) * (size_t)(M > 0 ? M : 1));
  for (int64_t q = 0; q < M; q++) {
    int64_t c[3];
    for (int d = 0; d < 3; d++) c[d] = wrap((int64_t)floor(X[d * M + q] / h), d == 2 ? Nz : N);
    int64_t nb = N / 8;
    int64_t blk = ((c[2] / 8) * nb + c[1] / 8) * nb + c[0] / 8;
    kv[q].key = (uint32_t)(((blk * 8 + c[2] % 8) * 8 + c[1] % 8) * 8 + c[0] % 8);
    kv[q].id = (int32_t)q;
  }
  qsort(kv, (size_t)M, sizeof(kv_t), kv_cmp);
  for (int64_t i = 0; i < M; i++) { keys_sorted[i] = kv[i].key; perm[i] = kv[i].id; }
  free(kv);
}

/* ------------------------------------------------------------------------
 * Material force (sub-step 1 of Sec. 3.2).  The paper defers fibre forces to
 * Peskin's review and shell forces to another work; the force laws below are
 * the reading used here, each the negative gradient of an energy:
 *   lattice stretch, edge (a,b):  E = 1/2 Ks kbar wbar (|d| - Le)^2 / Le^2,
 *       d = Xb - Xa, Le = |Yb - Ya|, kbar = (ka+kb)/2, wbar = (wa+wb)/2;
 *   lattice bend, triple (a,c,b): E = 1/2 Kb kc wc |D2X - D2Y|^2 / Lc^4,
 *       D2X = Xa - 2Xc + Xb, Lc = (|Yc - Ya| + |Yb - Yc|)/2;
 *   spring (a,b):                 E = 1/2 Ksp kbar (|d| - rest)^2;
 *   tether q:                     E = 1/2 kappa_q w_q |Xq - Yq|^2;
 * plus the window drive A w_q sin(2 pi f t) n_q (Sec. 4, oval window).
 * Y = X_ref.  Each marker's force is f(q) dq (area weight included).
 * With disp = 1 the state holds D = X - Y: an edge vector is formed as
 * (Yb - Ya) + (Db - Da), the bend's second difference as Da - 2Dc + Db and
 * the tether's offset as D itself (the same quantities, each with the
 * relative precision of the displacements).
 * ---------------------------------------------------------------------- */
static inline double norm3(const double v[3]) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

static void getp(const double *A, int64_t M, int64_t q, double out[3]) {
  out[0] = A[q]; out[1] = A[M + q]; out[2] = A[2 * M + q];
}

static void addp(double *A, int64_t M, int64_t q, const double v[3], double s) {
  A[q] += s * v[0]; A[M + q] += s * v[1]; A[2 * M + q] += s * v[2];
}

/* Edge vector Xb - Xa of the state X: positions (disp = 0), or
 * (Yb - Ya) + (Db - Da) from displacements D (disp = 1). */
static void edge_vec(const ibo_model *m, const double *X, int64_t a, int64_t b, double d[3]) {
  int64_t M = m->M;
  double xa[3], xb[3];
  getp(X, M, a, xa); getp(X, M, b, xb);
  if (m->disp) {
    double ya[3], yb[3];
    getp(m->X_ref, M, a, ya); getp(m->X_ref, M, b, yb);
    for (int i = 0; i < 3; i++) d[i] = (yb[i] - ya[i]) + (xb[i] - xa[i]);
  } else {
    for (int i = 0; i < 3; i++) d[i] = xb[i] - xa[i];
  }
}

/* Second difference from the reference, (Xa - 2Xc + Xb) - (Ya - 2Yc + Yb):
 * with displacements it is Da - 2Dc + Db. */
static void bend_vec(const ibo_model *m, const double *X, int64_t a, int64_t c, int64_t b, double v[3]) {
  int64_t M = m->M;
  double xa[3], xb[3], xc[3];
  getp(X, M, a, xa); getp(X, M, b, xb); getp(X, M, c, xc);
  if (m->disp) {
    for (int i = 0; i < 3; i++) v[i] = xa[i] - 2.0 * xc[i] + xb[i];
  } else {
    double ya[3], yb[3], yc[3];
    getp(m->X_ref, M, a, ya); getp(m->X_ref, M, b, yb); getp(m->X_ref, M, c, yc);
    for (int i = 0; i < 3; i++) v[i] = (xa[i] - 2.0 * xc[i] + xb[i]) - (ya[i] - 2.0 * yc[i] + yb[i]);
  }
}

void ibo_positions(const ibo_model *m, const double *X, double *P) {
  int64_t n3 = 3 * m->M;
  for (int64_t p = 0; p < n3; p++) P[p] = m->disp ? m->X_ref[p] + X[p] : X[p];
}

/* Extension |d| - Le of an edge whose reference vector is dy (Le = |dy|) and
 * current vector d.  From displacements (d = dy + dl, dl = Db - Da) it is
 * formed as (2 dy.dl + dl.dl) / (|d| + Le), the same number without the
 * cancellation of two lengths that agree to the strain. */
static double extension(const ibo_model *m, const double *X, int64_t a, int64_t b, const double dy[3],
                        const double d[3], double len, double Le) {
  if (!m->disp) return len - Le;
  int64_t M = m->M;
  double xa[3], xb[3], dl[3];
  getp(X, M, a, xa); getp(X, M, b, xb);
  for (int i = 0; i < 3; i++) dl[i] = xb[i] - xa[i];
  (void)d;
  double num = 2.0 * (dy[0] * dl[0] + dy[1] * dl[1] + dy[2] * dl[2]) + (dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
  return num / (len + Le);
}

/* Stretch edge: force added into F (if non-null), energy added into *E (if non-null). */
static void stretch_edge(const ibo_model *m, const double *X, int64_t a, int64_t b, double Ks,
                         int use_w, double *F, double *E) {
  int64_t M = m->M;
  double ya[3], yb[3], d[3], dy[3];
  getp(m->X_ref, M, a, ya); getp(m->X_ref, M, b, yb);
  edge_vec(m, X, a, b, d);
  for (int i = 0; i < 3; i++) dy[i] = yb[i] - ya[i];
  double len = norm3(d), Le = norm3(dy);
  double ext = extension(m, X, a, b, dy, d, len, Le);
  double K = Ks * 0.5 * (m->k[a] + m->k[b]);
  if (use_w) K *= 0.5 * (m->w[a] + m->w[b]);
  if (E) *E += 0.5 * K * ext * ext / (Le * Le);
  if (F) {
    /* dE/dXb = K (len - Le)/Le^2 * d/len ; dE/dXa = -dE/dXb */
    double s = K * ext / (Le * Le) / len;
    addp(F, M, a, d, s);
    addp(F, M, b, d, -s);
  }
}

static void bend_triple(const ibo_model *m, const double *X, int64_t a, int64_t c, int64_t b,
                        double Kb, double *F, double *E) {
  int64_t M = m->M;
  double ya[3], yb[3], yc[3], v[3], e1[3], e2[3];
  getp(m->X_ref, M, a, ya); getp(m->X_ref, M, b, yb); getp(m->X_ref, M, c, yc);
  bend_vec(m, X, a, c, b, v);
  for (int i = 0; i < 3; i++) {
    e1[i] = yc[i] - ya[i];
    e2[i] = yb[i] - yc[i];
  }
  double Lc = 0.5 * (norm3(e1) + norm3(e2));
  double K = Kb * m->k[c] * m->w[c] / (Lc * Lc * Lc * Lc);
  if (E) *E += 0.5 * K * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  if (F) {
    /* dE/dXa = K v, dE/dXc = -2 K v, dE/dXb = K v */
    addp(F, M, a, v, -K);
    addp(F, M, c, v, 2.0 * K);
    addp(F, M, b, v, -K);
  }
}

static void elastic_terms(const ibo_model *m, const double *X, double *F, double *E) {
  int64_t M = m->M;
  for (int l = 0; l < m->n_lat; l++) {
    int64_t f0 = m->lat_first[l];
    int64_t n1 = m->lat_n1[l], n2 = m->lat_n2[l];
    int per = m->lat_periodic2[l];
    double Ks = m->lat_Ks[l], Kb = m->lat_Kb[l];
#define IDX(i1, i2) (f0 + (int64_t)(i2) * n1 + (int64_t)(i1))
    if (Ks != 0.0) {
      for (int64_t i2 = 0; i2 < n2; i2++)
        for (int64_t i1 = 0; i1 + 1 < n1; i1++) stretch_edge(m, X, IDX(i1, i2), IDX(i1 + 1, i2), Ks, 1, F, E);
      int64_t e2 = per ? n2 : n2 - 1;
      for (int64_t i2 = 0; i2 < e2; i2++)
        for (int64_t i1 = 0; i1 < n1; i1++) stretch_edge(m, X, IDX(i1, i2), IDX(i1, (i2 + 1) % n2), Ks, 1, F, E);
    }
    if (Kb != 0.0) {
      for (int64_t i2 = 0; i2 < n2; i2++)
        for (int64_t i1 = 1; i1 + 1 < n1; i1++)
          bend_triple(m, X, IDX(i1 - 1, i2), IDX(i1, i2), IDX(i1 + 1, i2), Kb, F, E);
      for (int64_t i2 = 0; i2 < n2; i2++) {
        if (!per && (i2 == 0 || i2 == n2 - 1)) continue;
        for (int64_t i1 = 0; i1 < n1; i1++)
          bend_triple(m, X, IDX(i1, (i2 + n2 - 1) % n2), IDX(i1, i2), IDX(i1, (i2 + 1) % n2), Kb, F, E);
      }
    }
#undef IDX
  }
  for (int64_t e = 0; e < m->n_springs; e++) {
    int64_t a = m->spring_ab[e], b = m->spring_ab[m->n_springs + e];
    double d[3];
    edge_vec(m, X, a, b, d);
    double len = norm3(d), L0 = m->spring_rest[e];
    double K = m->K_spring * 0.5 * (m->k[a] + m->k[b]);
    if (E) *E += 0.5 * K * (len - L0) * (len - L0);
    if (F) {
      double s = K * (len - L0) / len;
      addp(F, M, a, d, s);
      addp(F, M, b, d, -s);
    }
  }
  if (m->kappa) {
    for (int64_t q = 0; q < M; q++) {
      double kw = m->kappa[q] * m->w[q];
      if (kw == 0.0) continue;
      double x[3], y[3], r[3];
      getp(X, M, q, x); getp(m->X_ref, M, q, y);
      for (int i = 0; i < 3; i++) r[i] = m->disp ? x[i] : x[i] - y[i];
      if (E) *E += 0.5 * kw * (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
      if (F) addp(F, M, q, r, -kw);
    }
  }
}

void ibo_force(const ibo_model *m, const double *X, double t, double *F) {
  int64_t M = m->M;
  memset(F, 0, sizeof(double) * 3 * (size_t)M);
  elastic_terms(m, X, F, NULL);
  if (m->n_drive > 0 && m->drive_A != 0.0) {
    double amp = m->drive_A * sin(2.0 * PI * m->drive_freq * t);
    for (int64_t j = 0; j < m->n_drive; j++) {
      int64_t q = m->drive_idx[j];
      double dir[3] = {m->drive_dir[j], m->drive_dir[m->n_drive + j], m->drive_dir[2 * m->n_drive + j]};
      addp(F, M, q, dir, amp * m->w[q]);
    }
  }
}

double ibo_energy(const ibo_model *m, const double *X) {
  double E = 0.0;
  elastic_terms(m, X, NULL, &E);
  return E;
}

/* ------------------------------------------------------------------------
 * Spreading, eq. discreteF (sub-step 2): F(x) = sum_q F_q delta_h(x - X_q),
 * F_q = f(q) dq.  delta_h vanishes unless |x_d - X_d| < 2h, so only the 4^3
 * nodes floor(X/h)-1 .. floor(X/h)+2 are visited; node indices wrap
 * periodically.  Plain scatter in marker order.
 *
 * Threads split the z-planes, not the markers: thread t of nt owns the
 * planes k with k mod nt = t, visits every marker in index order and adds
 * only into its own planes.  Each node therefore receives its terms in marker
 * order, as in a serial loop, and the result does not depend on the number
 * of threads.  The weight of node (i, j, k) is phi(s1 - i) phi(s2 - j)
 * phi(s3 - k) / h^3; the twelve factors are evaluated once per marker.
 * ---------------------------------------------------------------------- */
static void my_planes(int64_t *t, int64_t *nt) {
#ifdef _OPENMP
  *t = omp_get_thread_num();
  *nt = omp_get_num_threads();
#else
  *t = 0;
  *nt = 1;
#endif
}

/* phi(s - j) for the four nodes j = floor(s) - 1 .. floor(s) + 2 */
static void phi4(double s, int64_t c, double w[4]) {
  for (int a = 0; a < 4; a++) w[a] = ibo_phi(s - (double)(c - 1 + a));
}

void ibo_spread(int N, int Nz, double L, int64_t M, const double *X, const double *Fq, double *Fg) {
  int64_t G = (int64_t)N * N * Nz;
  double h = L / N, inv_h3 = 1.0 / (h * h * h);
  memset(Fg, 0, sizeof(double) * 3 * (size_t)G);
#pragma omp parallel
  {
    int64_t t, nt;
    my_planes(&t, &nt);
    for (int64_t q = 0; q < M; q++) {
      double s[3], w[3][4];
      int64_t c[3];
      for (int d = 0; d < 3; d++) { s[d] = X[d * M + q] / h; c[d] = (int64_t)floor(s[d]); }
      int mine = 0;
      for (int64_t k = c[2] - 1; k <= c[2] + 2; k++) mine |= wrap(k, Nz) % nt == t;
      if (!mine) continue;
      for (int d = 0; d < 3; d++) phi4(s[d], c[d], w[d]);
      for (int64_t k = c[2] - 1; k <= c[2] + 2; k++) {
        if (wrap(k, Nz) % nt != t) continue;
        for (int64_t j = c[1] - 1; j <= c[1] + 2; j++)
          for (int64_t i = c[0] - 1; i <= c[0] + 2; i++) {
            double dlt = w[0][i - c[0] + 1] * w[1][j - c[1] + 1] * w[2][k - c[2] + 1] * inv_h3;
            int64_t p = gidx(N, Nz, i, j, k);
            for (int cc = 0; cc < 3; cc++) Fg[cc * G + p] += Fq[cc * M + q] * dlt;
          }
      }
    }
  }
}

/* ------------------------------------------------------------------------
 * Interpolation, eq. discreteX (sub-step 4): U_q = sum_x u(x) delta_h(x - X_q) h^3
 * = sum over the same 4^3 nodes of u(x) phi phi phi.
 * ---------------------------------------------------------------------- */
void ibo_interp(int N, int Nz, double L, int64_t M, const double *X, const double *u, double *U) {
  int64_t G = (int64_t)N * N * Nz;
  double h = L / N;
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < M; q++) {
    double s[3], acc[3] = {0.0, 0.0, 0.0}, w[3][4];
    int64_t c[3];
    for (int d = 0; d < 3; d++) { s[d] = X[d * M + q] / h; c[d] = (int64_t)floor(s[d]); phi4(s[d], c[d], w[d]); }
    for (int64_t k = c[2] - 1; k <= c[2] + 2; k++)
      for (int64_t j = c[1] - 1; j <= c[1] + 2; j++)
        for (int64_t i = c[0] - 1; i <= c[0] + 2; i++) {
          double wgt = w[0][i - c[0] + 1] * w[1][j - c[1] + 1] * w[2][k - c[2] + 1];
          int64_t p = gidx(N, Nz, i, j, k);
          for (int cc = 0; cc < 3; cc++) acc[cc] += u[cc * G + p] * wgt;
        }
    for (int cc = 0; cc < 3; cc++) U[cc * M + q] = acc[cc];
  }
}

/* ------------------------------------------------------------------------
 * Upwind advection of eq. discreteNS1: for component c,
 *   A_c = sum_k u_k D_k^- u_c  (u_k > 0),  u_k D_k^+ u_c  (u_k < 0),  0 (u_k = 0),
 * with D^+ / D^- the one-sided differences of eqs. differenceOpsFirst-Last.
 * ---------------------------------------------------------------------- */
void ibo_advect(int N, int Nz, double L, const double *u, double *A) {
  int64_t G = (int64_t)N * N * Nz;
  double h = L / N;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < Nz; k++)
    for (int64_t j = 0; j < N; j++)
      for (int64_t i = 0; i < N; i++) {
        int64_t p = gidx(N, Nz, i, j, k);
        int64_t pm[3] = {gidx(N, Nz, i - 1, j, k), gidx(N, Nz, i, j - 1, k), gidx(N, Nz, i, j, k - 1)};
        int64_t pp[3] = {gidx(N, Nz, i + 1, j, k), gidx(N, Nz, i, j + 1, k), gidx(N, Nz, i, j, k + 1)};
        for (int c = 0; c < 3; c++) {
          const double *uc = u + c * G;
          double acc = 0.0;
          for (int kk = 0; kk < 3; kk++) {
            double uk = u[kk * G + p];
            if (uk > 0.0) acc += uk * ((uc[p] - uc[pm[kk]]) / h);
            else if (uk < 0.0) acc += uk * ((uc[pp[kk]] - uc[p]) / h);
          }
          A[c * G + p] = acc;
        }
      }
}

/* Transpose of the upwind advection linearised at u with each branch frozen
 * (the side taken by u_k(x) > 0, u_k(x) < 0 or neither is kept; R8):
 * the advection of ibo_advect is A_c(x) = sum_k u_k(x) D_k u_c(x), D_k the
 * backward difference where u_k(x) > 0 and the forward one where u_k(x) < 0,
 * so for a perturbation d,
 *   dA_c(x) = sum_k [ d_k(x) D_k u_c(x) + u_k(x) D_k d_c(x) ].
 * Written out for a cotangent r, out = (dA/du)^T r is, at each point y,
 *   out_k(y) = sum_c r_c(y) D_k u_c(y)                      (first term)
 *   out_c(y) += sum_k [ b_k(y) - b_k(y + e_k) - f_k(y) + f_k(y - e_k) ]
 * with b_k(x) = u_k(x) r_c(x) / h where u_k(x) > 0 (else 0) and
 * f_k(x) = u_k(x) r_c(x) / h where u_k(x) < 0 (else 0)    (second term). */
void ibo_advect_adjoint(int N, int Nz, double L, const double *u, const double *r, double *out) {
  int64_t G = (int64_t)N * N * Nz;
  double h = L / N;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < Nz; k++)
    for (int64_t j = 0; j < N; j++)
      for (int64_t i = 0; i < N; i++) {
        int64_t p = gidx(N, Nz, i, j, k);
        int64_t pm[3] = {gidx(N, Nz, i - 1, j, k), gidx(N, Nz, i, j - 1, k), gidx(N, Nz, i, j, k - 1)};
        int64_t pp[3] = {gidx(N, Nz, i + 1, j, k), gidx(N, Nz, i, j + 1, k), gidx(N, Nz, i, j, k + 1)};
        for (int c = 0; c < 3; c++) {
          const double *rc = r + c * G;
          double acc = 0.0;
          /* first term: component c receives sum_c' r_c'(y) D_c u_c'(y) */
          double uk = u[c * G + p];
          for (int cp = 0; cp < 3; cp++) {
            const double *ucp = u + cp * G;
            if (uk > 0.0) acc += r[cp * G + p] * ((ucp[p] - ucp[pm[c]]) / h);
            else if (uk < 0.0) acc += r[cp * G + p] * ((ucp[pp[c]] - ucp[p]) / h);
          }
          /* second term: the difference stencils of every direction k, transposed */
          for (int kk = 0; kk < 3; kk++) {
            const double *uk_ = u + kk * G;
            double at = uk_[p], up = uk_[pp[kk]], dn = uk_[pm[kk]];
            if (at > 0.0) acc += at * rc[p] / h;          /* b_k(y)        */
            if (up > 0.0) acc -= up * rc[pp[kk]] / h;     /* - b_k(y + e_k) */
            if (at < 0.0) acc -= at * rc[p] / h;          /* - f_k(y)      */
            if (dn < 0.0) acc += dn * rc[pm[kk]] / h;     /* f_k(y - e_k)  */
          }
          out[c * G + p] = acc;
        }
      }
}

/* ------------------------------------------------------------------------
 * FFT (named, not specified, in Sec. 3.2): an iterative radix-2
 * decimation-in-time transform of length n applied along each axis (the
 * plain DFT for a length that is not a power of two).
 * Twiddles exp(sign 2 pi i j / n) are evaluated directly with cos/sin.
 * ---------------------------------------------------------------------- */
static void fft1(int n, double *re, double *im, const double *cs, const double *sn, int sign) {
  for (int i = 1, j = 0; i < n; i++) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      double t = re[i]; re[i] = re[j]; re[j] = t;
      t = im[i]; im[i] = im[j]; im[j] = t;
    }
  }
  for (int len = 2; len <= n; len <<= 1) {
    int half = len / 2, step = n / len;
    for (int i0 = 0; i0 < n; i0 += len)
      for (int k = 0; k < half; k++) {
        double wr = cs[k * step], wi = sign * sn[k * step];
        int a = i0 + k, b = i0 + k + half;
        double xr = re[b] * wr - im[b] * wi;
        double xi = re[b] * wi + im[b] * wr;
        re[b] = re[a] - xr; im[b] = im[a] - xi;
        re[a] = re[a] + xr; im[a] = im[a] + xi;
      }
  }
}

/* A length that is not a power of two (a box whose z length carries a factor
 * 3): the DFT from its definition, X[k] = sum_j x[j] exp(sign 2 pi i j k / n),
 * with the angle's index j k taken mod n. */
static void dft1(int n, double *re, double *im, const double *cs, const double *sn, int sign, double *tr,
                 double *ti) {
  for (int k = 0; k < n; k++) {
    double ar = 0.0, ai = 0.0;
    for (int j = 0; j < n; j++) {
      int64_t e = ((int64_t)j * k) % n;
      double wr = cs[e], wi = sign * sn[e];
      ar += re[j] * wr - im[j] * wi;
      ai += re[j] * wi + im[j] * wr;
    }
    tr[k] = ar;
    ti[k] = ai;
  }
  for (int k = 0; k < n; k++) { re[k] = tr[k]; im[k] = ti[k]; }
}

void ibo_fft3(int N, int Nz, double *re, double *im, int sign) {
  int64_t NN = (int64_t)N * N, G = NN * Nz;
  for (int axis = 0; axis < 3; axis++) {
    int n = axis == 2 ? Nz : N;                    /* transform length along this axis */
    int64_t stride = axis == 0 ? 1 : (axis == 1 ? N : NN);
    int64_t npen = G / n;
    double *cs = (double *)malloc(sizeof(double) * n), *sn = (double *)malloc(sizeof(double) * n);
    for (int j = 0; j < n; j++) { cs[j] = cos(2.0 * PI * j / n); sn[j] = sin(2.0 * PI * j / n); }
#pragma omp parallel
    {
      double *br = (double *)malloc(sizeof(double) * n), *bi = (double *)malloc(sizeof(double) * n);
      double *tr = (double *)malloc(sizeof(double) * n), *ti = (double *)malloc(sizeof(double) * n);
      const int pow2 = (n & (n - 1)) == 0;
#pragma omp for schedule(static)
      for (int64_t pencil = 0; pencil < npen; pencil++) {
        /* pencil enumerates the two other axes */
        int64_t a = pencil % N, b = pencil / N, base;
        if (axis == 0) base = b * NN + a * N;          /* (j=a, k=b) */
        else if (axis == 1) base = b * NN + a;         /* (i=a, k=b) */
        else base = b * N + a;                         /* (i=a, j=b) */
        for (int t = 0; t < n; t++) { br[t] = re[base + t * stride]; bi[t] = im[base + t * stride]; }
        if (pow2) fft1(n, br, bi, cs, sn, sign);
        else dft1(n, br, bi, cs, sn, sign, tr, ti);
        for (int t = 0; t < n; t++) { re[base + t * stride] = br[t]; im[base + t * stride] = bi[t]; }
      }
      free(br); free(bi); free(tr); free(ti);
    }
    free(cs); free(sn);
  }
}

/* ------------------------------------------------------------------------
 * Navier-Stokes update, eqs. discreteNS1-2 (sub-step 3).  With
 *   r = u^n - dt sum_k u_k D_k^{+-} u^n + (dt/rho) F^n,
 * the system reads (I - (mu dt/rho) sum_k D+_k D-_k) u' + (dt/rho) D0 p = r,
 * D0 . u' = 0.  In Fourier mode m the symbols are
 *   sum_k D+_k D-_k -> -lambda,  lambda = sum_d (4/h^2) sin^2(pi m_d / N_d),
 *   D0_d            -> i s_d,    s_d    = sin(2 pi m_d / N_d) / h,
 * (N_d the nodes along axis d: N, N, Nz), so w = r^/(1 + (mu dt/rho) lambda)
 * and u'^ = w - s (s.w)/|s|^2, or u'^ = w when s = 0 (every m_d in
 * {0, N_d/2}: D0 annihilates the mode, no pressure).
 * ---------------------------------------------------------------------- */
static double sin_mode(int m, int N) {
  /* sin(2 pi m / N), exactly 0 at m = 0 and m = N/2 where the true value is 0 */
  if (m == 0 || 2 * m == N) return 0.0;
  return sin(2.0 * PI * (double)m / (double)N);
}

double ibo_fluid(int N, int Nz, double L, double rho, double mu, double dt, int convect,
                 const double *u, const double *Fg, double *u_new) {
  int64_t G = (int64_t)N * N * Nz;
  double h = L / N;
  double *re = (double *)malloc(sizeof(double) * 3 * (size_t)G);
  double *im = (double *)calloc(3 * (size_t)G, sizeof(double));
  double *A = NULL;
  if (convect) {
    A = (double *)malloc(sizeof(double) * 3 * (size_t)G);
    ibo_advect(N, Nz, L, u, A);
  }
  for (int64_t p = 0; p < 3 * G; p++) {
    double r = u[p];
    if (convect) r = r - dt * A[p];
    if (Fg) r = r + (dt / rho) * Fg[p];
    re[p] = r;
  }
  free(A);
  for (int c = 0; c < 3; c++) ibo_fft3(N, Nz, re + c * G, im + c * G, -1);

  double nu_dt = mu * dt / rho;
#pragma omp parallel for schedule(static)
  for (int64_t m3 = 0; m3 < Nz; m3++)
    for (int64_t m2 = 0; m2 < N; m2++)
      for (int64_t m1 = 0; m1 < N; m1++) {
        int64_t p = (m3 * N + m2) * N + m1;
        int64_t mm[3] = {m1, m2, m3};
        double lam = 0.0, s[3];
        for (int d = 0; d < 3; d++) {
          int nd = d == 2 ? Nz : N;       /* modes along z are those of period Nz */
          double sh = sin(PI * (double)mm[d] / (double)nd);
          lam += (4.0 / (h * h)) * sh * sh;
          s[d] = sin_mode((int)mm[d], nd) / h;
        }
        double den = 1.0 + nu_dt * lam;
        double wr[3], wi[3];
        for (int c = 0; c < 3; c++) { wr[c] = re[c * G + p] / den; wi[c] = im[c * G + p] / den; }
        double ss = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
        if (ss > 0.0) {
          double dr = (s[0] * wr[0] + s[1] * wr[1] + s[2] * wr[2]) / ss;
          double di = (s[0] * wi[0] + s[1] * wi[1] + s[2] * wi[2]) / ss;
          for (int c = 0; c < 3; c++) { wr[c] -= s[c] * dr; wi[c] -= s[c] * di; }
        }
        for (int c = 0; c < 3; c++) { re[c * G + p] = wr[c]; im[c * G + p] = wi[c]; }
      }

  for (int c = 0; c < 3; c++) ibo_fft3(N, Nz, re + c * G, im + c * G, +1);
  double inv = 1.0 / (double)G, maxre = 0.0, maxim = 0.0;
  for (int64_t p = 0; p < 3 * G; p++) {
    u_new[p] = re[p] * inv;
    if (fabs(u_new[p]) > maxre) maxre = fabs(u_new[p]);
    if (fabs(im[p] * inv) > maxim) maxim = fabs(im[p] * inv);
  }
  free(re); free(im);
  return maxre > 0.0 ? maxim / maxre : maxim;
}

/* ------------------------------------------------------------------------
 * One time step, in the order of the enumerated list of Sec. 3.2:
 * force f^n, spread to F^n, NS update to u^{n+1}, move markers with u^{n+1}
 * interpolated at X^n (eq. discreteX).
 * ---------------------------------------------------------------------- */
void ibo_step(const ibo_model *m, int N, int Nz, double L, double rho, double mu, double dt,
              int convect, double t, double *X, double *u, double *F_lag_out) {
  int64_t M = m->M, G = (int64_t)N * N * Nz;
  double *F = (double *)malloc(sizeof(double) * 3 * (size_t)(M > 0 ? M : 1));
  double *Fg = (double *)malloc(sizeof(double) * 3 * (size_t)G);
  double *un = (double *)malloc(sizeof(double) * 3 * (size_t)G);
  double *U = (double *)malloc(sizeof(double) * 3 * (size_t)(M > 0 ? M : 1));
  double *P = (double *)malloc(sizeof(double) * 3 * (size_t)(M > 0 ? M : 1));
  ibo_positions(m, X, P);   /* where the delta function is evaluated */
  ibo_force(m, X, t, F);
  if (F_lag_out) memcpy(F_lag_out, F, sizeof(double) * 3 * (size_t)M);
  ibo_spread(N, Nz, L, M, P, F, Fg);
  ibo_fluid(N, Nz, L, rho, mu, dt, convect, u, Fg, un);
  ibo_interp(N, Nz, L, M, P, un, U);
  for (int64_t p = 0; p < 3 * M; p++) X[p] = X[p] + dt * U[p];
  memcpy(u, un, sizeof(double) * 3 * (size_t)G);
  free(F); free(Fg); free(un); free(U); free(P);
}

/* ------------------------------------------------------------------------
 * Adjoint (reverse mode) of one step with convect = 0.  Not in the paper: it
 * differentiates the four sub-steps above.  Writing Phi_q(x) =
 * phi(s1-i)phi(s2-j)phi(s3-k) (s = X_q/h), the forward step is
 *   f = force(X^n),  F = S f = sum_q f_q Phi_q / h^3,  r = u^n + (dt/rho) F,
 *   u' = Lop r  (Lop = the linear NS update above, symmetric),
 *   X' = X^n + dt sum_x u'(x) Phi_q(x).
 * Given Xbar', ubar' the adjoints at n are
 *   Ubar = dt Xbar';  Xbar = Xbar' + sum_x (u'(x).Ubar_q) dPhi_q/dX_q;
 *   ubar_tot = ubar' + sum_q Ubar_q Phi_q;  rbar = Lop ubar_tot;  ubar^n = rbar;
 *   Fbar = (dt/rho) rbar;  fbar_q = sum_x Fbar(x) Phi_q / h^3;
 *   Xbar += sum_x (Fbar(x).f_q) dPhi_q/dX_q / h^3;  Xbar += (df/dX)^T fbar;
 *   kbar += (df/dk)^T fbar,
 * with dPhi_q/dX_{q,d} = phi'(s_d - j_d)/h * (product of the other two phi).
 * ---------------------------------------------------------------------- */
static double dphi(double r) {
  /* derivative of phi; phi is even, so phi' is odd */
  double a = fabs(r), g;
  if (a <= 1.0) g = (-2.0 + (4.0 - 8.0 * a) / (2.0 * sqrt(1.0 + 4.0 * a - 4.0 * a * a))) / 8.0;
  else if (a <= 2.0) {
    double b = 2.0 - a; /* phi(a) = 1/2 - phi(b), d/da = +phi'(b) */
    g = (-2.0 + (4.0 - 8.0 * b) / (2.0 * sqrt(1.0 + 4.0 * b - 4.0 * b * b))) / 8.0;
  } else g = 0.0;
  return r < 0.0 ? -g : g;
}

/* phi(s - j) and phi'(s - j) / h for the four nodes j = floor(s) - 1 .. floor(s) + 2 */
static void phi4_d(double s, int64_t c, double h, double w[4], double g[4]) {
  for (int a = 0; a < 4; a++) {
    double r = s - (double)(c - 1 + a);
    w[a] = ibo_phi(r);
    g[a] = dphi(r) / h;
  }
}

/* One edge term E = 1/2 Ku kf (|d| - L0)^2 / D, D = L0^2 (rest_sq) or 1, with
 * d = Xb - Xa, Ku the stiffness at unit k-factor and kf the k-factor.
 * Adds H v into out and returns f_unit . v, the force of the edge at unit
 * k-factor dotted with v.  dE/dd = K'(1 - L0/|d|) d, K' = Ku kf / D, and
 * d2E/dd2 = K' [(1 - L0/|d|) I + (L0/|d|^3) d d^T]. */
static double hess_edge(const ibo_model *m, const double *X, int64_t a, int64_t b, double Ku,
                        double kf, double L0, int rest_sq, const double *v, double *out) {
  int64_t M = m->M;
  double d[3], va[3], vb[3], dv[3];
  edge_vec(m, X, a, b, d);
  getp(v, M, a, va); getp(v, M, b, vb);
  for (int i = 0; i < 3; i++) dv[i] = vb[i] - va[i];
  double len = norm3(d);
  /* |d| - L0: for a lattice edge (rest length |Yb - Ya|) from displacements as in the force */
  double ext = len - L0;
  if (rest_sq) {
    double ya[3], yb[3], dy[3];
    getp(m->X_ref, M, a, ya); getp(m->X_ref, M, b, yb);
    for (int i = 0; i < 3; i++) dy[i] = yb[i] - ya[i];
    ext = extension(m, X, a, b, dy, d, len, L0);
  }
  double Ku_p = rest_sq ? Ku / (L0 * L0) : Ku;
  double Kp = Ku_p * kf;
  double dd = d[0] * dv[0] + d[1] * dv[1] + d[2] * dv[2];
  double Hv[3];
  for (int i = 0; i < 3; i++) Hv[i] = Kp * ((ext / len) * dv[i] + (L0 / (len * len * len)) * dd * d[i]);
  addp(out, M, b, Hv, 1.0);
  addp(out, M, a, Hv, -1.0);
  /* unit force: -c d at b, +c d at a, c = Ku'(|d| - L0)/|d|; dotted with v: -c d.(vb - va) */
  return -(Ku_p * ext / len) * dd;
}

static void elastic_hvp_and_kbar(const ibo_model *m, const double *X, const double *v,
                                 double *Hv, double *kbar) {
  int64_t M = m->M;
  for (int l = 0; l < m->n_lat; l++) {
    int64_t f0 = m->lat_first[l];
    int64_t n1 = m->lat_n1[l], n2 = m->lat_n2[l];
    int per = m->lat_periodic2[l];
    double Ks = m->lat_Ks[l], Kb = m->lat_Kb[l];
#define IDX(i1, i2) (f0 + (int64_t)(i2) * n1 + (int64_t)(i1))
    if (Ks != 0.0) {
      int64_t e2 = per ? n2 : n2 - 1;
      for (int dir = 0; dir < 2; dir++)
        for (int64_t i2 = 0; i2 < (dir == 0 ? n2 : e2); i2++)
          for (int64_t i1 = 0; i1 < (dir == 0 ? n1 - 1 : n1); i1++) {
            int64_t a = IDX(i1, i2), b = dir == 0 ? IDX(i1 + 1, i2) : IDX(i1, (i2 + 1) % n2);
            double ya[3], yb[3], dy[3];
            getp(m->X_ref, M, a, ya); getp(m->X_ref, M, b, yb);
            for (int i = 0; i < 3; i++) dy[i] = yb[i] - ya[i];
            double Le = norm3(dy);
            double kb = 0.5 * (m->k[a] + m->k[b]), wb = 0.5 * (m->w[a] + m->w[b]);
            /* kbar_e = (k_a + k_b)/2, so df/dk_a = df/dk_b = 1/2 (edge force at unit kbar_e) */
            double gdv = hess_edge(m, X, a, b, Ks * wb, kb, Le, 1, v, Hv);
            kbar[a] += 0.5 * gdv;
            kbar[b] += 0.5 * gdv;
          }
    }
    if (Kb != 0.0) {
      for (int dir = 0; dir < 2; dir++)
        for (int64_t i2 = 0; i2 < n2; i2++)
          for (int64_t i1 = 0; i1 < n1; i1++) {
            int64_t a, c, b;
            if (dir == 0) {
              if (i1 == 0 || i1 == n1 - 1) continue;
              a = IDX(i1 - 1, i2); c = IDX(i1, i2); b = IDX(i1 + 1, i2);
            } else {
              if (!per && (i2 == 0 || i2 == n2 - 1)) continue;
              a = IDX(i1, (i2 + n2 - 1) % n2); c = IDX(i1, i2); b = IDX(i1, (i2 + 1) % n2);
            }
            double ya[3], yb[3], yc[3], e1[3], e2v[3], z[3], vv[3];
            getp(m->X_ref, M, a, ya); getp(m->X_ref, M, b, yb); getp(m->X_ref, M, c, yc);
            double va[3], vb[3], vc[3];
            getp(v, M, a, va); getp(v, M, b, vb); getp(v, M, c, vc);
            bend_vec(m, X, a, c, b, vv);
            for (int i = 0; i < 3; i++) {
              e1[i] = yc[i] - ya[i]; e2v[i] = yb[i] - yc[i];
              z[i] = va[i] - 2.0 * vc[i] + vb[i];
            }
            double Lc = 0.5 * (norm3(e1) + norm3(e2v));
            double K1 = Kb * m->w[c] / (Lc * Lc * Lc * Lc); /* per unit k_c */
            double K = K1 * m->k[c];
            addp(Hv, M, a, z, K);
            addp(Hv, M, c, z, -2.0 * K);
            addp(Hv, M, b, z, K);
            /* force at unit k_c: -K1 vv at a and b, +2 K1 vv at c; dotted with v */
            kbar[c] += -K1 * (vv[0] * z[0] + vv[1] * z[1] + vv[2] * z[2]);
          }
    }
#undef IDX
  }
  for (int64_t e = 0; e < m->n_springs; e++) {
    int64_t a = m->spring_ab[e], b = m->spring_ab[m->n_springs + e];
    double kb = 0.5 * (m->k[a] + m->k[b]);
    double gdv = hess_edge(m, X, a, b, m->K_spring, kb, m->spring_rest[e], 0, v, Hv);
    kbar[a] += 0.5 * gdv;
    kbar[b] += 0.5 * gdv;
  }
  if (m->kappa)
    for (int64_t q = 0; q < M; q++) {
      double kw = m->kappa[q] * m->w[q];
      if (kw == 0.0) continue;
      double vq[3];
      getp(v, M, q, vq);
      addp(Hv, M, q, vq, kw);
    }
}

void ibo_adjoint_step(const ibo_model *m, int N, int Nz, double L, double rho, double mu, double dt,
                      double t, const double *X_n, const double *u_np1,
                      double *Xbar, double *ubar, double *kbar) {
  ibo_adjoint_step_u(m, N, Nz, L, rho, mu, dt, t, 0, X_n, NULL, u_np1, Xbar, ubar, kbar);
}

void ibo_adjoint_step_u(const ibo_model *m, int N, int Nz, double L, double rho, double mu, double dt,
                        double t, int convect, const double *X_n, const double *u_n, const double *u_np1,
                        double *Xbar, double *ubar, double *kbar) {
  int64_t M = m->M, G = (int64_t)N * N * Nz;
  double h = L / N, inv_h3 = 1.0 / (h * h * h);
  size_t mb = sizeof(double) * 3 * (size_t)(M > 0 ? M : 1);
  double *f = (double *)malloc(mb), *Ub = (double *)malloc(mb), *fb = (double *)calloc(3 * (size_t)(M > 0 ? M : 1), sizeof(double));
  double *Hv = (double *)calloc(3 * (size_t)(M > 0 ? M : 1), sizeof(double));
  double *utot = (double *)malloc(sizeof(double) * 3 * (size_t)G);
  double *Pn = (double *)malloc(mb);
  ibo_positions(m, X_n, Pn);   /* the delta function's arguments at step n */
  ibo_force(m, X_n, t, f);
  for (int64_t p = 0; p < 3 * M; p++) Ub[p] = dt * Xbar[p];

  /* interpolation: phi' term into Xbar (a gather per marker) */
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < M; q++) {
    double s[3];
    int64_t c[3];
    for (int d = 0; d < 3; d++) { s[d] = Pn[d * M + q] / h; c[d] = (int64_t)floor(s[d]); }
    double gX[3] = {0.0, 0.0, 0.0}, w[3][4], g[3][4];
    for (int d = 0; d < 3; d++) phi4_d(s[d], c[d], h, w[d], g[d]);
    for (int64_t k = c[2] - 1; k <= c[2] + 2; k++)
      for (int64_t j = c[1] - 1; j <= c[1] + 2; j++)
        for (int64_t i = c[0] - 1; i <= c[0] + 2; i++) {
          int a0 = (int)(i - c[0] + 1), a1 = (int)(j - c[1] + 1), a2 = (int)(k - c[2] + 1);
          double p0 = w[0][a0], p1 = w[1][a1], p2 = w[2][a2];
          double g0 = g[0][a0], g1 = g[1][a1], g2 = g[2][a2];
          int64_t p = gidx(N, Nz, i, j, k);
          double uU = 0.0;
          for (int cc = 0; cc < 3; cc++) uU += u_np1[cc * G + p] * Ub[cc * M + q];
          gX[0] += uU * g0 * p1 * p2;
          gX[1] += uU * p0 * g1 * p2;
          gX[2] += uU * p0 * p1 * g2;
        }
    for (int d = 0; d < 3; d++) Xbar[d * M + q] += gX[d];
  }
  /* and its transpose, a spread without 1/h^3, into utot (z-planes dealt
   * to threads as in ibo_spread: every node sums in marker order) */
  memcpy(utot, ubar, sizeof(double) * 3 * (size_t)G);
#pragma omp parallel
  {
    int64_t t, nt;
    my_planes(&t, &nt);
    for (int64_t q = 0; q < M; q++) {
      double s[3], w[3][4];
      int64_t c[3];
      for (int d = 0; d < 3; d++) { s[d] = Pn[d * M + q] / h; c[d] = (int64_t)floor(s[d]); }
      int mine = 0;
      for (int64_t k = c[2] - 1; k <= c[2] + 2; k++) mine |= wrap(k, Nz) % nt == t;
      if (!mine) continue;
      for (int d = 0; d < 3; d++) phi4(s[d], c[d], w[d]);
      for (int64_t k = c[2] - 1; k <= c[2] + 2; k++) {
        if (wrap(k, Nz) % nt != t) continue;
        for (int64_t j = c[1] - 1; j <= c[1] + 2; j++)
          for (int64_t i = c[0] - 1; i <= c[0] + 2; i++) {
            double wgt = w[0][i - c[0] + 1] * w[1][j - c[1] + 1] * w[2][k - c[2] + 1];
            int64_t p = gidx(N, Nz, i, j, k);
            for (int cc = 0; cc < 3; cc++) utot[cc * G + p] += Ub[cc * M + q] * wgt;
          }
      }
    }
  }

  /* symmetric NS operator (no force, no advection) */
  ibo_fluid(N, Nz, L, rho, mu, dt, 0, utot, NULL, ubar);

  /* spreading: transpose (an interpolation with 1/h^3) and phi' term, per marker */
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < M; q++) {
    double s[3];
    int64_t c[3];
    for (int d = 0; d < 3; d++) { s[d] = Pn[d * M + q] / h; c[d] = (int64_t)floor(s[d]); }
    double gX[3] = {0.0, 0.0, 0.0}, acc[3] = {0.0, 0.0, 0.0}, w[3][4], g[3][4];
    for (int d = 0; d < 3; d++) phi4_d(s[d], c[d], h, w[d], g[d]);
    for (int64_t k = c[2] - 1; k <= c[2] + 2; k++)
      for (int64_t j = c[1] - 1; j <= c[1] + 2; j++)
        for (int64_t i = c[0] - 1; i <= c[0] + 2; i++) {
          int a0 = (int)(i - c[0] + 1), a1 = (int)(j - c[1] + 1), a2 = (int)(k - c[2] + 1);
          double p0 = w[0][a0], p1 = w[1][a1], p2 = w[2][a2];
          double g0 = g[0][a0], g1 = g[1][a1], g2 = g[2][a2];
          int64_t p = gidx(N, Nz, i, j, k);
          double Ff = 0.0;
          for (int cc = 0; cc < 3; cc++) {
            double Fb = (dt / rho) * ubar[cc * G + p];
            Ff += Fb * f[cc * M + q];
            acc[cc] += Fb * (p0 * p1 * p2) * inv_h3;
          }
          gX[0] += Ff * g0 * p1 * p2 * inv_h3;
          gX[1] += Ff * p0 * g1 * p2 * inv_h3;
          gX[2] += Ff * p0 * p1 * g2 * inv_h3;
        }
    for (int d = 0; d < 3; d++) { Xbar[d * M + q] += gX[d]; fb[d * M + q] = acc[d]; }
  }

  /* force: Xbar += (df/dX)^T fbar = -H fbar ; kbar += (df/dk)^T fbar */
  elastic_hvp_and_kbar(m, X_n, fb, Hv, kbar);
  for (int64_t p = 0; p < 3 * M; p++) Xbar[p] -= Hv[p];

  /* ubar is the cotangent of r = u - dt A(u) + (dt / rho) F; with advection
   * the velocity's own adjoint loses dt (dA/du)^T rbar */
  if (convect) {
    ibo_advect_adjoint(N, Nz, L, u_n, ubar, utot);
    for (int64_t p = 0; p < 3 * G; p++) ubar[p] -= dt * utot[p];
  }

  free(f); free(Ub); free(fb); free(Hv); free(utot); free(Pn);
}
