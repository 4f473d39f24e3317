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
constexpr int kLatPre = 12;       // reference-shape constants per lattice marker (see k_lattice_pre)
constexpr int kTile = 8;          // cells per tile edge: markers are binned by 8^3-cell tiles
constexpr int kHalo = 11;         // nodes per edge of a tile's stencil halo (cells -1 .. 9)
constexpr int kHalo3 = kHalo * kHalo * kHalo;
constexpr int kPartStride = 4096;  // values per item halo: 3 * 11^3, padded so that 64 lanes copy it in whole rounds

// Sorted marker record (fluid precision): fractional offset s - floor(s) per
// dimension, the spread force (or, in the adjoint, the staged dt * Xbar), and
// the cell key.  16-byte aligned so a record is a few vector loads.
template <typename T>
struct Rec;
template <>
struct alignas(16) Rec<float> {
  float f[3];
  uint32_t key;
  float F[3];
  int pad;
};
template <>
struct alignas(16) Rec<double> {
  double f[3];
  double F[3];
  uint32_t key;
  int pad[3];
};

// Cell key (binning of Sec. 3.3): cells are grouped in 8^3 tiles;
// key = tile * 512 + (lz * 8 + ly) * 8 + lx with l the cell within the tile and
// tile = (tz * nt + ty) * nt + tx, nt = n / 8 (tz < nz / 8).  A tile's
// markers are one contiguous run of the sorted order.
__host__ __device__ __forceinline__ uint32_t cell_key(int cx, int cy, int cz, int log2nt) {
  const uint32_t tile = ((uint32_t)(cz >> 3) << (2 * log2nt)) | ((uint32_t)(cy >> 3) << log2nt) | (uint32_t)(cx >> 3);
  return (tile << 9) | ((uint32_t)(cz & 7) << 6) | ((uint32_t)(cy & 7) << 3) | (uint32_t)(cx & 7);
}
// A cell (or node) index wrapped periodically into [0, len), len any positive
// length (the z length need not be a power of two).
__host__ __device__ __forceinline__ int wrap_cell(int64_t c, int len) {
  const int64_t r = c % len;
  return (int)(r < 0 ? r + len : r);
}

// Position of a cell's stencil origin (node cell - 1) in its tile's 11^3 halo.
__host__ __device__ __forceinline__ int halo_base(uint32_t key) {
  return (int)((key >> 6) & 7) * (kHalo * kHalo) + (int)((key >> 3) & 7) * kHalo + (int)(key & 7);
}

// Work items: the sorted markers are cut into chunks of `chunk` markers (one
// per spreading wave) and into tiles; an item is the part of one tile that
// lies in one chunk.  Item j of tile t (markers [ts, te)) covers
// [max(ts, (ts / chunk + j) chunk), min(te, (ts / chunk + j + 1) chunk)).
__device__ __forceinline__ void item_range(int item, const int32_t *__restrict__ tile_start,
                                           const int32_t *__restrict__ tile_item0,
                                           const int32_t *__restrict__ item_tile, int chunk, int *j0, int *j1) {
  const int tile = item_tile[item];
  const int ts = tile_start[tile], te = tile_start[tile + 1];
  const int cj = ts / chunk + (item - tile_item0[tile]);
  *j0 = max(ts, cj * chunk);
  *j1 = min(te, (cj + 1) * chunk);
}

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
  // reference-shape constants of the lattices, [kLatPre][M] (see k_lattice_pre), or null
  const double *lat_pre;
  // 1: marker state arrays hold displacements D = X - X_ref (ib_params.displacement)
  int32_t disp;
};

// Device-side state of the binning: full sort this call, movers listed,
// some mover changed tile, range [lo, hi] of sorted positions that change.
enum BinState { BS_FULL = 0, BS_NMOV = 1, BS_TILES = 2, BS_LO = 3, BS_HI = 4, BS_WORDS = 8 };
constexpr int kMoverCap = 4096;   // most movers the incremental update takes (one block sorts them)
// The movers' list, kMoverCap entries per array: as listed (id, new key, old
// sorted position), then sorted by (new key, id) (key, id, new position) and
// the old positions and old keys, ascending.
enum MoverList { MV_Q = 0, MV_KEY, MV_POS, MS_KEY, MS_VAL, MS_NEW, MS_OLD, MS_OLDKEY, MV_ARRAYS };

struct Workspace {
  // binning
  uint32_t *keys[2];
  int32_t *vals[2];
  uint32_t *keys_id;           // [M] cell key of each marker at the last binning
  uint32_t *bin_state;         // [BS_WORDS] the binning's device-side state (BinState)
  int32_t *bin_mov;            // [MV_ARRAYS][kMoverCap] the movers' list (MoverList)
  uint32_t *hist;
  int nblk_sort;
  int32_t *tile_start;         // [ntiles + 1] first sorted position of each tile
  int32_t *inv;                // [M] sorted position of each marker
  // sorted marker records (fluid precision)
  void *recs;                  // [M] Rec<T>
  double *Flag;                // [3][M] force workspace (f64)
  double *fb;                  // [3][M] adjoint force cotangent (f64)
  // grid
  void *Fgrid;                 // [3][G] spread force density
  // work list: items = the parts of the tiles within the chunks
  int32_t *tile_nit;           // [ntiles] work items of the tile
  int32_t *tile_item0;         // [ntiles] first work item of the tile
  int32_t *tile_touch;         // [ntiles] 1 if the spread force reaches the tile (dense in Fgrid), else 0
  uint32_t *touch_bits;        // [ceil(ntiles / 32)] the same flags, bit t & 31 of word t >> 5
  int32_t *item_tile;          // [item_cap] tile of each work item
  int32_t *chunk_item0;        // [nchunks + 1] first item of each chunk; the last entry = items
  int32_t *nitems;             // [3] work items, split tiles, touched tiles
  int32_t *split_list;         // [ntiles] tiles with more than one item
  int32_t *touch_list;         // [ntiles] tiles the spread force reaches
  int32_t *scan_tmp;           // [3 ceil(ntiles / 1024)] per-block scan totals
  void *partials;              // [item_cap][kPartStride] each item's spread halo, [3][11^3] + pad
  void *r;                     // [3][G] right-hand side (radix-2 path only; null for n = 32 .. 256)
  void *spec;                  // [3][n/2+1][nz][n] complex spectrum
  int32_t *nonfinite;          // [1] flag for checked mode
  // tables (fluid precision): along x and y of length n, along z of length nz
  void *tw;                    // [n] complex exp(-2 pi i k / n)
  void *lam;                   // [n] (4/h^2) sin^2(pi m / n)
  void *sgrad;                 // [n] sin(2 pi m / n) / h (exact 0 at m = 0, n/2)
  void *twz, *lamz, *sgradz;   // the same for length nz
  // drive
  int32_t *drive_idx;          // [D]
  double *drive_dir;           // [3][D]
  int32_t *drive_slot;         // [M] index into the drive list, -1 if not driven (null when D = 0)
  // spring adjacency
  int32_t *sp_rowptr, *sp_col;
  double *sp_rest;
  double *lat_pre;             // [kLatPre][M] lattice reference constants (null without lattice moduli)
};

// Phases timed by the optional HIP-event instrumentation.
enum Phase {
  PH_BIN = 0, PH_FORCE, PH_PREP, PH_SPREAD, PH_SPLIT, PH_GATHER, PH_RHS, PH_FFT_X, PH_FFT_Y, PH_FFT_Z_SOLVE,
  PH_FFT_Y_INV, PH_FFT_X_INV, PH_INTERP, PH_ADJ_INTERP, PH_ADJ_SPREAD, PH_HESSVEC, PH_RHS_FFT_X, PH_ADJ_ADVECT,
  PH_FFT_YX_INV, PH_COUNT
};

struct TimerRec {
  int phase;
  hipEvent_t a, b;
};

}  // namespace ib

struct ib_ctx {
  ib_params p;
  int n = 0, log2n = 0;
  int nz = 0;               // nodes along z: n (cube), n / 2 (half-cube) or 3 n / 4
  int64_t G = 0, M = 0;     // G = n * n * nz
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
  bool bin_reuse = true;   // keep the last partition when no marker changed cell
  int log2nt = 0;       // log2(n / 8)
  int ntz = 0;          // nz / 8 (tiles along z)
  int64_t ntiles = 0;
  int ncu = 256;        // compute units of the device
  int item_grid = 0;    // most single-wave blocks of the spreading kernel
  int chunk = 1;        // markers per chunk (per spreading wave)
  int nchunks = 0;
  int64_t item_cap = 0;
  // instrumentation
  bool timing = false;
  uint32_t tmask = 0xFFFFFFFFu;   // phases that record events while timing
  bool tskip = false;             // the open phase is not timed
  std::vector<ib::TimerRec> trec;
  size_t tused = 0;
  double tms[ib::PH_COUNT] = {};
  int64_t tcalls[ib::PH_COUNT] = {};
  // HIP graph of ib_step (ib_graph_enable): captured on cap_stream for one set of
  // (X, u, F_lag_out) pointers, replayed on `stream` with the force kernel's
  // drive amplitude updated per step
  bool graph_on = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipGraphNode_t graph_force = nullptr;      // the force kernel's node (null when M = 0)
  hipKernelNodeParams graph_force_params{};
  std::vector<void *> graph_force_args;      // its argument pointers, the amplitude's pointing at graph_amp
  double graph_amp = 0.0;
  const void *graph_key[3] = {nullptr, nullptr, nullptr};
  int64_t graph_captures = 0, graph_launches = 0;
};

namespace ib {

// ---- launchers (each returns hipError_t of the launch) ----
hipError_t launch_bin(ib_ctx *c, const double *X);   // -> keys/vals[sorted_buf], inv, tile_start, work list
hipError_t launch_force(ib_ctx *c, const double *X, double amp, double *F);
// force and the sorted records in one pass (needs the binning); F nullable
template <typename T>
hipError_t launch_force_rec(ib_ctx *c, const double *X, double amp, double *F);
// the kernel launch_force_rec launches, and the position of `amp` among its arguments
// (for updating a captured launch)
template <typename T>
const void *force_rec_kernel(bool disp);
constexpr int kForceRecAmpArg = 5;
constexpr int kForceRecArgs = 13;
template <typename T>
hipError_t launch_prep(ib_ctx *c, const double *X, const double *F);      // sorted records
template <typename T>
hipError_t launch_spread(ib_ctx *c, T *Fgrid, bool dense_zero, double scale);  // -> Fgrid, tile_touch
// r = u - dt A(u) [convect] + f_scale F; fmode 0: no F, 1: F in marked tiles, 2: dense F
template <typename T>
hipError_t launch_rhs(ib_ctx *c, const T *u, const T *Fgrid, int fmode, int convect, double f_scale, T *r);
template <typename T>
hipError_t launch_fluid_solve(ib_ctx *c, const T *r, T *u_out);           // FFT, solve, iFFT
// The whole NS update u_out = Lop(u_in - dt A(u_in) [convect] + f_scale F): register
// FFT passes for n in {32, 64, 128, 256}, otherwise launch_rhs + launch_fluid_solve.
bool fluid_reg_supported(int n, int nz);
template <typename T>
hipError_t launch_fluid_reg(ib_ctx *c, const T *u_in, const T *Fg, int fmode, int convect, double f_scale,
                            T *u_out);
template <typename T>
hipError_t launch_fluid(ib_ctx *c, const T *u_in, const T *Fg, int fmode, int convect, double f_scale, T *u_out);
// U = S*(X_pos) u (FP64 weights and sums); X_inout += dt U when given, U_out = U when given
template <typename T>
hipError_t launch_interp(ib_ctx *c, const T *u, const double *X_pos, double *X_inout, double *U_out, double dt);

// adjoint pieces
template <typename T>
hipError_t launch_adj_interp(ib_ctx *c, const T *u_np1, const double *X_n, double *Xbar);   // stages dt*Xbar in recs[].F
template <typename T>
hipError_t launch_adj_spread(ib_ctx *c, const T *ubar_n, const double *F, const double *X_n, double *Xbar,
                             double *fbar);
hipError_t launch_hessvec(ib_ctx *c, const double *X, const double *v, double *Xbar, double *kbar);
// reference-shape constants of the lattices from X_ref and w (at creation and when they are set)
hipError_t launch_lattice_pre(ib_ctx *c);
hipError_t launch_probe(ib_ctx *c, const double *X, const double *X0, const int32_t *idx, const double *dir,
                        int64_t count, double *disp, double *env);
// adjoint step with advection: ubar -= dt (dA/du)^T ubar at u^n (tmp: [3][G] scratch)
template <typename T>
hipError_t launch_adv_adjoint(ib_ctx *c, const T *u_n, const T *rbar, T *ubar);   // ubar = rbar - dt A'^T rbar

// text returned by ib_last_error(NULL)
void set_context_free_error(const std::string &msg);

// instrumentation: event pair around a phase when timing is on
void timer_begin(ib_ctx *c, int phase);
void timer_end(ib_ctx *c);
struct PhaseScope {
  ib_ctx *c;
  PhaseScope(ib_ctx *ctx, int phase) : c(ctx) { timer_begin(c, phase); }
  ~PhaseScope() { timer_end(c); }
};

}  // namespace ib
