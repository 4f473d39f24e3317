/*
 * ibo.h -- ORACLE for the immersed-boundary (IB) time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct FP64 CPU
 * implementation of what the GPU library computes.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may call it; the
 * product path never does.  It shares no code, header, table or helper with
 * the GPU library.
 *
 * Source: E. Givelberg and J. Bunn, "A Comprehensive Three-Dimensional Model
 * of the Cochlea", Sec. 3 (the immersed boundary method):
 *   - the four sub-steps of one time step (Sec. 3.2, enumerated list);
 *   - difference operators D+_i, D-_i, D0_i (eqs. differenceOpsFirst-Last);
 *   - the discrete Navier-Stokes system with upwind advection
 *     (eqs. discreteNS1, discreteNS2), solved by FFT (Sec. 3.2);
 *   - force spreading (eq. discreteF) and interpolation/move (eq. discreteX);
 *   - the 4-point function phi and delta_h (Sec. 3.2, end);
 *   - the marker/grid partitioning of Sec. 3.3 (here: a cell-key binning).
 * Readings where the paper is silent are listed in the repository's design
 * notes; the ones that change arithmetic are restated next to the code.
 *
 * Layouts: marker arrays are SoA [3][M] (component-major); grid arrays are
 * [3][Nz][N][N] with x fastest: element (c, k, j, i) at ((c*Nz + k)*N + j)*N + i,
 * grid node (i, j, k) at position (i h, j h, k h), h = L / N.  The box is
 * L x L x (Nz h): Nz = N is the cube, Nz = N/2 the half-cube of Sec. 4.
 * Every function taking (N, Nz) wraps x and y with period N, z with Nz.
 */
#ifndef IBO_H
#define IBO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* phi(r) of Sec. 3.2; delta_h(x) = h^-3 phi(x1/h) phi(x2/h) phi(x3/h). */
double ibo_phi(double r);

/* Binning: cell of marker q is c_d = floor(X_d / h) wrapped into [0, N)
 * ([0, Nz) along z; N, Nz multiples of 8); with block
 * b = ((c3/8) (N/8) + c2/8) (N/8) + c1/8,
 * key = ((b * 8 + c3%8) * 8 + c2%8) * 8 + c1%8.  perm lists marker ids ordered
 * by key, ties by marker id (a stable sort).  keys_sorted[i] = key of perm[i]. */
void ibo_bin(int N, int Nz, double L, int64_t M, const double *X,
             uint32_t *keys_sorted, int32_t *perm);

/* Material force F_q = f(q) dq on every marker (sub-step 1), and its energy. */
typedef struct {
  int64_t M;
  const double *w, *k, *X_ref, *kappa;          /* [M], [M], [3][M], [M]   */
  int32_t n_lat;
  const int64_t *lat_first;                     /* [n_lat]                 */
  const int32_t *lat_n1, *lat_n2, *lat_periodic2;
  const double *lat_Ks, *lat_Kb;
  int64_t n_springs;
  const int32_t *spring_ab;                     /* [2][S]                  */
  const double *spring_rest;                    /* [S]                     */
  double K_spring;
  int64_t n_drive;
  const int32_t *drive_idx;                     /* [D]                     */
  const double *drive_dir;                      /* [3][D]                  */
  double drive_A, drive_freq;
  /* 0: marker arrays hold positions X.  1: they hold displacements D = X - Y
   * from the reference shape Y = X_ref; positions are formed as Y + D where
   * the delta function is evaluated, and the elastic terms are written in D
   * (an edge is (Yb - Ya) + (Db - Da), a second difference Da - 2Dc + Db), so
   * that strains far below the positions' rounding keep their own relative
   * precision. */
  int32_t disp;
} ibo_model;

void   ibo_force(const ibo_model *m, const double *X, double t, double *F);
double ibo_energy(const ibo_model *m, const double *X);

/* Positions Y + D of a model's markers whose state array holds displacements
 * (disp = 1); copies X when disp = 0.  P: [3][M]. */
void ibo_positions(const ibo_model *m, const double *X, double *P);

/* Sub-step 2, eq. discreteF: Fg = sum_q F_q delta_h(x - X_q) (overwrite). */
void ibo_spread(int N, int Nz, double L, int64_t M, const double *X, const double *Fq, double *Fg);
/* Sub-step 4 velocity, eq. discreteX: U_q = sum_x u(x) delta_h(x - X_q) h^3. */
void ibo_interp(int N, int Nz, double L, int64_t M, const double *X, const double *u, double *U);
/* Upwind advection sum_k u_k D_k^{+-} u (eq. discreteNS1), [3][G] -> [3][G], G = N^2 Nz. */
void ibo_advect(int N, int Nz, double L, const double *u, double *A);
/* out = (dA/du)^T r: the transpose of ibo_advect linearised at u, each
 * upwind branch frozen at the sign u_k(x) takes. */
void ibo_advect_adjoint(int N, int Nz, double L, const double *u, const double *r, double *out);
/* In-place complex 3-D DFT of an Nz x N x N array (x fastest): sign -1
 * forward, +1 inverse; no normalisation. */
void ibo_fft3(int N, int Nz, double *re, double *im, int sign);
/* Sub-step 3, eqs. discreteNS1-2: u_new from u, Fg.  Returns the largest
 * |imaginary part| of the inverse transform relative to max |u_new|. */
double ibo_fluid(int N, int Nz, double L, double rho, double mu, double dt, int convect,
                 const double *u, const double *Fg, double *u_new);
/* One full time step: X, u advanced in place; F_lag_out (nullable) gets f^n dq. */
void ibo_step(const ibo_model *m, int N, int Nz, double L, double rho, double mu, double dt,
              int convect, double t, double *X, double *u, double *F_lag_out);

/* Reverse-mode (adjoint) step for convect = 0, given Xbar, ubar at n+1:
 * overwrites them with the adjoints at n and accumulates kbar += (df/dk)^T fbar. */
void ibo_adjoint_step(const ibo_model *m, int N, int Nz, double L, double rho, double mu, double dt,
                      double t, const double *X_n, const double *u_np1,
                      double *Xbar, double *ubar, double *kbar);
/* The same for either convect setting; u_n (the step's starting velocity,
 * where the upwind branches are frozen) is read when convect = 1. */
void ibo_adjoint_step_u(const ibo_model *m, int N, int Nz, double L, double rho, double mu, double dt,
                        double t, int convect, const double *X_n, const double *u_n, const double *u_np1,
                        double *Xbar, double *ubar, double *kbar);

int ibo_num_threads(void);
/* Threads of the parallel loops from here on (nt > 0); results do not depend on it. */
void ibo_set_num_threads(int nt);

#ifdef __cplusplus
}
#endif
#endif
