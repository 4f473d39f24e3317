// Internal declarations of the IB library: the context, its workspace, and
// the launchers of every kernel.  Device code for gfx950 (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ib.h"

namespace ib {

constexpr int kMaxLattices = 16;
constexpr int kTile = 8;          // spreading tile: 8^3 grid nodes per block
constexpr int kSpreadItem = 1024; // most markers one spreading work item takes

// Sorted marker record (fluid precision): fractional offset s - floor(s) per
// dimension, the spread force (or, in the adjoint, the staged dt * Xbar), and
// the cell's x index.  16-byte aligned so a record is a few vector loads.
template <typename T>
struct Rec;
template <>
struct alignas(16) Rec<float> {
  float f[3];
  int cx;
  float F[3];
  int pad;
};
template <>
struct alignas(16) Rec<double> {
  double f[3];
  double F[3];
  int cx;
  int pad[3];
};

struct LatticeDev {
  int64_t first;
  int32_t n1, n2, periodic2;
  double Ks, Kb;
};

struct LatticeTable {
  int32_t n;
  LatticeDev l[kMaxLattices];
};

// Pointers of the per-marker material model used by the force kernels.
struct Material {
  const double *w, *k, *X_ref, *kappa;
  LatticeTable lat;
  const int32_t *sp_rowptr;   // [M+1] spring adjacency (CSR), or null
  const int32_t *sp_col;      // [2S]
  const double *sp_rest;      // [2S]
  double K_spring;
  int64_t M;
};

struct Workspace {
  // binning
  uint32_t *keys[2];
  int32_t *vals[2];
  uint32_t *hist;
  int nblk_sort;
  int32_t *row_start;          // [n^2 + 1]
  // sorted marker records (fluid precision)
  void *recs;                  // [M] Rec<T>
  double *Flag;                // [3][M] force workspace (f64)
  double *fb;                  // [3][M] adjoint force cotangent (f64)
  // grid
  void *Fgrid;                 // [3][G] spread force density
  // spreading work list (8^3 tiles)
  int32_t *rowtab;             // [n^2][2 (n/8 + 1)] row boundary positions
  int32_t *tile_count;         // [ntiles] markers listed per tile
  int32_t *tile_flag;          // [ntiles] work items of the tile (0: no force; else dense in Fgrid)
  int32_t *tile_part;          // [ntiles] first partial of a split tile
  int32_t *tile_item0;         // [ntiles] first work item of the tile
  int32_t *item_tile;          // [item_cap] tile of each work item
  int32_t *nitems;             // [3] work items, split tiles, next item to take
  int32_t *split_list;         // [ntiles] tiles with more than one item
  int32_t *scan_tmp;           // [3 * ceil(ntiles / 1024)] per-block scan totals
  void *partials;              // [part_cap][3][512] partial tiles of split tiles
  void *r;                     // [3][G] right-hand side
  void *spec;                  // [3][n/2+1][n][n] complex spectrum
  int32_t *nonfinite;          // [1] flag for checked mode
  // tables (fluid precision)
  void *tw;                    // [n/2] complex exp(-2 pi i k / n)
  void *lam;                   // [n] (4/h^2) sin^2(pi m / n)
  void *sgrad;                 // [n] sin(2 pi m / n) / h (exact 0 at m = 0, n/2)
  // drive
  int32_t *drive_idx;          // [D]
  double *drive_dir;           // [3][D]
  // spring adjacency
  int32_t *sp_rowptr, *sp_col;
  double *sp_rest;
};

// Phases timed by the optional HIP-event instrumentation.
enum Phase {
  PH_BIN = 0, PH_FORCE, PH_PREP, PH_SPREAD, PH_RHS, PH_FFT_X, PH_FFT_Y, PH_FFT_Z_SOLVE, PH_FFT_Y_INV,
  PH_FFT_X_INV, PH_INTERP, PH_ADJ_INTERP, PH_ADJ_SPREAD, PH_HESSVEC, PH_COUNT
};

struct TimerRec {
  int phase;
  hipEvent_t a, b;
};

}  // namespace ib

struct ib_ctx {
  ib_params p;
  int n = 0, log2n = 0;
  int64_t G = 0, M = 0;
  double h = 0.0;
  bool fp32 = false;
  bool check = false;
  hipStream_t stream = nullptr;
  std::string err;
  ib::Material mat{};
  int64_t n_springs = 0, n_drive = 0;
  double drive_A = 0.0, drive_freq = 0.0;
  ib::Workspace ws{};
  int64_t ws_bytes = 0;
  int sort_passes = 0, digit_bits = 0;
  int sorted_buf = 0;   // which keys/vals buffer holds the sorted result
  int spread_grid = 0;  // blocks of the persistent spreading kernel
  int64_t item_cap = 0, part_cap = 0;
  // instrumentation
  bool timing = false;
  std::vector<ib::TimerRec> trec;
  size_t tused = 0;
  double tms[ib::PH_COUNT] = {};
  int64_t tcalls[ib::PH_COUNT] = {};
};

namespace ib {

// ---- launchers (each returns hipError_t of the launch) ----
hipError_t launch_bin(ib_ctx *c, const double *X);   // -> keys/vals[sorted_buf], row_start
hipError_t launch_force(ib_ctx *c, const double *X, double amp, double *F);
template <typename T>
hipError_t launch_prep(ib_ctx *c, const double *X, const double *F);      // sorted records
template <typename T>
hipError_t launch_spread(ib_ctx *c, T *Fgrid, bool dense_zero, double scale);  // -> Fgrid, tile_flag
// r = u - dt A(u) [convect] + f_scale F; fmode 0: no F, 1: F in marked tiles, 2: dense F
template <typename T>
hipError_t launch_rhs(ib_ctx *c, const T *u, const T *Fgrid, int fmode, int convect, double f_scale, T *r);
template <typename T>
hipError_t launch_fluid_solve(ib_ctx *c, const T *r, T *u_out);           // FFT, solve, iFFT
// The whole NS update u_out = Lop(u_in - dt A(u_in) [convect] + f_scale F): register
// FFT passes for n in {32, 64, 128, 256}, otherwise launch_rhs + launch_fluid_solve.
bool fluid_reg_supported(int n);
template <typename T>
hipError_t launch_fluid_reg(ib_ctx *c, const T *u_in, const T *Fg, int fmode, int convect, double f_scale,
                            T *u_out);
template <typename T>
hipError_t launch_fluid(ib_ctx *c, const T *u_in, const T *Fg, int fmode, int convect, double f_scale, T *u_out);
template <typename T>
hipError_t launch_interp(ib_ctx *c, const T *u, double *X_inout, double *U_out, double dt);

// adjoint pieces
template <typename T>
hipError_t launch_adj_interp(ib_ctx *c, const T *u_np1, double *Xbar);   // stages dt*Xbar in recs[].F
template <typename T>
hipError_t launch_adj_spread(ib_ctx *c, const T *ubar_n, const double *F, double *Xbar, double *fbar);
hipError_t launch_hessvec(ib_ctx *c, const double *X, const double *v, double *Xbar, double *kbar);

// instrumentation: event pair around a phase when timing is on
void timer_begin(ib_ctx *c, int phase);
void timer_end(ib_ctx *c);
struct PhaseScope {
  ib_ctx *c;
  PhaseScope(ib_ctx *ctx, int phase) : c(ctx) { timer_begin(c, phase); }
  ~PhaseScope() { timer_end(c); }
};

}  // namespace ib
