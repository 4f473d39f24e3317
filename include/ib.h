/*
 * ib.h -- immersed-boundary (IB) time step on one AMD Instinct MI355X (gfx950).
 *
 * Implements the first-order IB scheme of Givelberg & Bunn, "A Comprehensive
 * Three-Dimensional Model of the Cochlea", Sec. 3.2: per step (1) the material
 * force f^n, (2) spreading F^n = sum_q f^n(q) delta_h(x - X^n(q)) dq
 * (eq. discreteF), (3) the Navier-Stokes update of eqs. discreteNS1-2 on a
 * periodic grid by FFT, (4) the marker move of eq. discreteX.  The adjoint
 * step is not in the paper; it differentiates the same four sub-steps.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grid: a periodic box of n x n x nz nodes at positions (i h, j h, k h),
 *    h = L/n (one mesh width in all directions; n a power of two in
 *    [8, 512]).  nz = n is the cube; nz = n/2 is the half-cube of Sec. 4
 *    (box L x L x L/2), available for n in [32, 256].
 *  - Grid fields (u, F_grid, ubar) are DEVICE arrays [3][nz][n][n], x fastest:
 *    component c of node (i, j, k) at ((c*nz + k)*n + j)*n + i, in the fluid
 *    precision (double for IB_FLUID_FP64, float for IB_FLUID_FP32).
 *  - Marker arrays (X, F_lag, U, Xbar) are DEVICE double arrays [3][M]
 *    (component-major).  X is stored unwrapped; only grid indices wrap.
 *    With ib_params.displacement = 1 every marker-state argument (the X of
 *    ib_step, ib_force, ib_spread, ib_interp, ib_bin, ib_adjoint_step(_u)
 *    and ib_probe) holds D = X - X_ref instead: positions are formed as
 *    X_ref + D where the delta function is evaluated, and the elastic terms
 *    from D (an edge as (Yb - Ya) + (Db - Da), a second difference as
 *    Da - 2Dc + Db, a tether offset as D), so that strains far below the
 *    rounding of O(1) positions keep their relative precision.  The move is
 *    D += dt U; Xbar is the same cotangent in both forms.
 *  - Per-marker forces are f(q) dq, i.e. force densities times the marker's
 *    area weight (so sum_x F_grid h^3 = sum_q F_lag[q]).
 *  - The caller owns every array it passes; the context owns only its
 *    workspace.  Calls are asynchronous on the context's stream: arrays must
 *    stay valid until that stream's work is done.  With the environment
 *    variable IB_CHECK=1 every call synchronises and checks for errors.
 *  - Errors are returned as IB_E* codes (never abort, never throw);
 *    ib_last_error() gives a text.  A context is not thread-safe.
 */
#ifndef IB_H
#define IB_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ib_ctx ib_ctx;

enum {
  IB_OK = 0,
  IB_EINVAL = -1,      /* bad argument (size, pointer, parameter out of range)   */
  IB_ENOMEM = -2,      /* device allocation failed                                */
  IB_EDEVICE = -3,     /* HIP runtime / kernel launch error                       */
  IB_ENOTSUP = -4,     /* valid request outside what this library supports        */
  IB_ENONFINITE = -5   /* IB_CHECK=1 found a NaN or Inf in an output              */
};

enum { IB_FLUID_FP64 = 0, IB_FLUID_FP32 = 1 };  /* markers are always FP64 */

/* Problem statement of Sec. 3.1-3.2: density rho, viscosity mu, periodic grid,
 * time step dt.  convect = 1 keeps the upwind advection term of
 * eq. discreteNS1, 0 drops it (a Stokes step; required by the adjoint). */
typedef struct {
  int32_t n;                 /* nodes per dimension: power of two, 8..512          */
  double L;                  /* box edge (> 0); h = L / n                           */
  double rho, mu, dt;        /* rho > 0, mu >= 0, dt > 0                            */
  int32_t fluid_precision;   /* IB_FLUID_FP64 or IB_FLUID_FP32                      */
  int32_t convect;           /* 0 or 1                                               */
  int64_t n_markers;         /* M >= 0, < 2^31                                      */
  void *stream;              /* hipStream_t (NULL: the null stream)                 */
  int32_t nz;                /* nodes along z: 0 or n (cube), n/2 (half-cube)       */
  int32_t displacement;      /* 0: marker arrays X hold positions; 1: they hold     */
                             /* displacements D = X - X_ref (see below)             */
} ib_params;

/* A rectangular material lattice Q (Sec. 3.2): markers first + i2*n1 + i1,
 * i1 in [0,n1) fastest, i2 in [0,n2) (periodic when periodic2 != 0). */
typedef struct {
  int64_t first;
  int32_t n1, n2, periodic2;
  double Ks, Kb;             /* stretch and bend moduli (0: term off)               */
} ib_lattice;

/* The material model (sub-step 1).  The paper defers fibre and shell forces
 * to other works; the laws used here are negative energy gradients:
 *   lattice stretch, edge (a,b): 1/2 Ks kbar wbar (|Xb-Xa| - |Yb-Ya|)^2 / |Yb-Ya|^2
 *   lattice bend, triple (a,c,b): 1/2 Kb k_c w_c |(Xa-2Xc+Xb) - (Ya-2Yc+Yb)|^2 / Lc^4,
 *       Lc = (|Yc-Ya| + |Yb-Yc|)/2
 *   spring (a,b): 1/2 K_spring kbar (|Xb-Xa| - rest)^2
 *   tether q:     1/2 kappa_q w_q |Xq - Yq|^2
 *   drive (window, Sec. 4): + drive_A w_q sin(2 pi drive_freq t) dir_q
 * with kbar, wbar the means over the edge's two markers and Y = X_ref.
 * w, k, X_ref, kappa are DEVICE arrays read at every call (the caller may
 * change their contents between calls; ib_set_material swaps pointers),
 * except that the lattice rest lengths |Yb-Ya|, Lc, the reference second
 * differences Ya - 2Yc + Yb and the factors wbar, w_c
 * are derived from X_ref and w once, at ib_create and at every
 * ib_set_material that passes w or X_ref: after changing the contents of
 * either in place, call ib_set_material with it again.
 * Topology (lattices, springs, drive) is HOST memory copied at ib_create. */
typedef struct {
  const double *w;           /* [M] area weight dq                                  */
  const double *k;           /* [M] stiffness multiplier (stretch, bend, springs)   */
  const double *X_ref;       /* [3][M] reference shape: tether targets, rest shape  */
  const double *kappa;       /* [M] tether stiffness density, 0 = none; nullable    */
  int32_t n_lattices;        /* <= 16                                               */
  const ib_lattice *lattices;
  int64_t n_springs;
  const int32_t *spring_ab;  /* [2][S] marker pairs (host)                          */
  const double *spring_rest; /* [S] rest lengths (host)                             */
  double K_spring;
  int64_t n_drive;
  const int32_t *drive_idx;  /* [D] distinct driven markers (host)                  */
  const double *drive_dir;   /* [3][D] drive directions (host)                      */
  double drive_A, drive_freq;
} ib_elastic;

/* Validate, copy the topology, allocate the workspace.  IB_EINVAL on a bad
 * parameter or topology index, IB_ENOTSUP for n outside [8, 512] or not a
 * power of two, or nz other than 0, n and n/2 (n/2 only for n in [32, 256]),
 * IB_ENOMEM on allocation failure, IB_EINVAL for displacement other than 0,
 * 1.  *out is NULL on error. */
int ib_create(const ib_params *p, const ib_elastic *e, ib_ctx **out);
void ib_destroy(ib_ctx *c);

/* Replace the per-marker material pointers (NULL keeps the current one).
 * Passing w or X_ref (even the same pointer) recomputes the lattice
 * constants derived from them, on the context's stream. */
int ib_set_material(ib_ctx *c, const double *w, const double *k, const double *X_ref,
                    const double *kappa);
/* Run subsequent calls on another hipStream_t. */
int ib_set_stream(ib_ctx *c, void *stream);

/* One time step (Sec. 3.2, all four sub-steps) at time t = n dt: X^n -> X^{n+1}
 * and u^n -> u^{n+1} in place.  F_lag_out (nullable, [3][M] double) receives
 * f^n dq.  Markers move with u^{n+1} interpolated at X^n (eq. discreteX). */
int ib_step(ib_ctx *c, double *X, void *u, double t, double *F_lag_out);

/* Replay ib_step as a HIP graph (the computation loop of Sec. 3.3 repeats the
 * same launches every step).  While on, the first ib_step with a given
 * (X, u, F_lag_out) triple captures the step's kernel launches (on an internal
 * stream; nothing runs during the capture) into a graph, and every ib_step
 * with the same three pointers launches that graph on the context's stream,
 * with only the force kernel's drive amplitude A sin(2 pi f t) updated; other
 * pointers capture anew.  ib_set_material drops the graph (it holds the
 * material pointers).  Results are bitwise those of the launches without the
 * graph.  Bypassed while the timers are enabled or IB_CHECK=1.  on = 0 drops
 * the graph.  Capture or launch failures are IB_EDEVICE. */
int ib_graph_enable(ib_ctx *c, int on);
/* Graphs captured and launched on this context so far. */
int ib_graph_stats(const ib_ctx *c, int64_t *captures, int64_t *launches);

/* Update of the marker partition (Sec. 3.3 partitions the material points
 * among the processors; here binning orders them by 8^3-cell tile and cell).
 * With on = 1 (the default) every binning compares each marker's cell with
 * the one it had at the last binning: with no change the sorted order, tile
 * ranges and work list stay; with up to 4096 markers in new cells those are
 * moved into place in the last sorted order (the work list is rebuilt only
 * if one changed tile); with more, or on the first binning, the markers are
 * sorted in full.  The choice is made on the device, so no call waits for
 * the host.  on = 0 sorts in full at every binning.  The results are bitwise
 * the same either way.  on other than 0 or 1: IB_EINVAL. */
int ib_bin_reuse(ib_ctx *c, int on);

/* Sub-step 1: F_lag = f(X, t) dq, [3][M] double (overwritten). */
int ib_force(ib_ctx *c, const double *X, double t, double *F_lag);

/* Sub-step 2, eq. discreteF: F_grid = sum_q F_lag[q] delta_h(x - X_q)
 * (overwrites the whole [3][nz][n][n] F_grid). */
int ib_spread(ib_ctx *c, const double *X, const double *F_lag, void *F_grid);

/* Velocity of eq. discreteX: U_q = sum_x u(x) delta_h(x - X_q) h^3, [3][M] double. */
int ib_interp(ib_ctx *c, const double *X, const void *u, double *U);

/* Sub-step 3, eqs. discreteNS1-2: u^n -> u^{n+1} in place given F_grid
 * (nullable: no body force). */
int ib_fluid(ib_ctx *c, void *u, const void *F_grid);

/* ib_fluid without a context, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Reads n, nz, L, rho, mu, dt, fluid_precision, convect and
 * stream from *p (n_markers is ignored) and updates u^n -> u^{n+1} in place
 * given F_grid (nullable: no body force), as ib_fluid does, on that stream.
 * Its spectrum and tables live in a static device array of 32 MiB that every
 * GPU the library runs on holds until the process ends; it calls no device
 * allocator.  Sizes: n in {32, 64, 128, 256}, nz in {0, n, n/2}, and the
 * spectrum, 3 (n/2+1) n nz complex values in the fluid precision, plus the
 * tables within 32 MiB (FP32: up to 128^3 and 128 x 128 x 64; FP64: up to
 * 64^3 and 128 x 128 x 64); IB_ENOTSUP for larger grids, IB_EINVAL for bad
 * parameters, IB_EDEVICE on a launch failure, the text in ib_last_error(NULL).
 * Calls on one GPU share the array: calls that overlap on one GPU (other
 * streams, other threads) race. */
int ib_fluid_noalloc(const ib_params *p, void *u, const void *F_grid);

/* The binning that partitions markers among grid cells (Sec. 3.3): the cell
 * of marker q is c = floor(X_q / h) per dimension wrapped into [0, n) ([0, nz)
 * along z); cells are grouped in 8^3 tiles,
 * tile = ((c3/8)*(n/8) + c2/8)*(n/8) + c1/8, and
 * key = tile*512 + ((c3%8)*8 + c2%8)*8 + c1%8.  perm[i] lists marker ids by
 * key, ties by id (stable); keys_sorted[i] is the key of perm[i].  Both
 * DEVICE arrays of length M. */
int ib_bin(ib_ctx *c, const double *X, uint32_t *keys_sorted, int32_t *perm);

/* Adjoint of ib_step for convect = 0 (IB_ENOTSUP otherwise).  Inputs: X_n
 * (the step's starting positions), u_np1 (the velocity it produced), t.
 * On entry Xbar [3][M] double and ubar [3][nz][n][n] (fluid precision) hold the
 * adjoints at step n+1; on return they hold those at step n, and
 * kbar [M] double has (df/dk)^T fbar added to it. */
int ib_adjoint_step(ib_ctx *c, const double *X_n, const void *u_np1, double t,
                    double *Xbar, void *ubar, double *kbar);
/* The same for either convect setting.  With convect = 1 the upwind advection
 * of eq. discreteNS1 is differentiated with each branch frozen at the side
 * u^n selects (the derivative away from u_k = 0; no term where u_k = 0), so
 * u_n [3][nz][n][n] (fluid precision, the velocity the step started from) is
 * required; with convect = 0 it is not read and may be NULL.  IB_EINVAL when
 * it is missing for convect = 1. */
int ib_adjoint_step_u(ib_ctx *c, const double *X_n, const void *u_n, const void *u_np1, double t,
                      double *Xbar, void *ubar, double *kbar);

/* Diagnostics of Sec. 5 (the membrane's displacement along its length and
 * its envelope over time): for i < count, the displacement of marker idx[i]
 * from X0 along the unit direction dir[:, i],
 *   disp[i] = sum_c (X[c][idx[i]] - X0[c][idx[i]]) dir[c][i],
 * and env[i] = max(env[i], |disp[i]|).  X, X0 [3][M] and dir [3][count]
 * double, idx [count] int32, disp and env [count] double (either NULL): all
 * DEVICE arrays.  An index outside [0, M) gives disp[i] = NaN and leaves
 * env[i].  IB_EINVAL for count < 0 or a missing X, X0, idx, dir. */
int ib_probe(ib_ctx *c, const double *X, const double *X0, const int32_t *idx, const double *dir,
             int64_t count, double *disp, double *env);

/* Text of the last error on this context ("" if none); c may be NULL for the
 * last error of ib_create or ib_fluid_noalloc on this thread. */
const char *ib_last_error(const ib_ctx *c);

/* Device bytes held by the context's workspace. */
int64_t ib_workspace_bytes(const ib_ctx *c);

/* Per-phase timing (the instrumentation of Sec. 3.3, here with HIP events on
 * the context's stream).  While enabled, every phase of every call records a
 * start/stop event pair; ib_timers_read synchronises the stream and returns,
 * for phase i < min(max, IB_N_TIMERS), the summed milliseconds ms[i] and the
 * number of launches calls[i] since the last reset.  Phase names come from
 * ib_timer_name(i) (NULL past the last phase).  Enabling resets the sums. */
#define IB_N_TIMERS 32
int ib_timers_enable(ib_ctx *c, int on);
/* Restrict the timed phases to those whose bit (1u << i) is set in mask (all
 * phases by default); each timed phase adds two events to the stream.  Phases
 * are numbered below IB_N_TIMERS, so every one has a bit in the mask. */
int ib_timers_select(ib_ctx *c, uint32_t mask);
int ib_timers_read(ib_ctx *c, double *ms, int64_t *calls, int max);
const char *ib_timer_name(int i);

#ifdef __cplusplus
}
#endif
#endif
