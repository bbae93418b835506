// Kernel argument blocks and launcher declarations shared by the host library.
#pragma once
#include "common.hpp"

namespace petto {

enum SweepMode { kSweep = 0, kCheck = 1, kResid = 2, kRefine = 3 };

// Geometry and boundary description of one elastic design.
struct ElGeom {
  int nx, ny, nz;           // cells per axis (nz = 1 in 2D)
  int px, py;               // padded extents nx+1, ny+1
  long plane;               // elements of one padded component array
  double h;
  double lam0, mu0;         // Lame parameters at unit modulus (Eq. 3.10)
  int clamp[6];             // side is clamped: tangential unknowns reflect, edges active
  int fixn[6];              // side holds the normal unknown at zero (clamped or roller)
  const uint32_t* pins;     // extra Dirichlet unknowns as a bitmask, or nullptr
  int tile3d;               // 3D sweep tiling: 1 large columns, 2 small columns
};

template <typename T>
struct ElSweep {
  const T* uin;             // state read (ping)
  T* uout;                  // state written (pong); residual mode: unused
  T* v;                     // velocity, updated in place; residual mode: receives r
  T* vout;                  // multi-sweep kernels: velocity written here (windows read
                            // their neighbours' halo velocities, so no in-place update)
  const T* E;               // cell modulus
  const T* b;               // right-hand side per unknown (force units)
  const SolveState* st;     // coefficients and stop flag (sweep / check; refine: stop flag or nullptr)
  double* partial;          // per-tile sum of r^2 (check / refine modes)
  float* b32;               // refine: receives float(r)
};

// Launchers return the number of tiles (= partial-sum slots written).
template <typename T, int MODE>
int launch_el2d(const ElGeom& g, const ElSweep<T>& a, hipStream_t s);
template <typename T, int MODE>
int launch_el3d(const ElGeom& g, const ElSweep<T>& a, hipStream_t s);
int el2d_tiles(const ElGeom& g);
int el3d_tiles(const ElGeom& g);   // the largest tile count of every precision and tiling
// K sweeps per launch on an LDS window (K in {2, 4, 5, 8, 10}); bit-identical to K
// launches of the one-sweep kernel.  CHECK: the last sweep also sums r^2.
template <typename T, int K, bool CHECK>
int launch_el2d_tb(const ElGeom& g, const ElSweep<T>& a, hipStream_t s);
int el2d_tb_tiles(const ElGeom& g, int K);   // 0 for an unsupported K
int el3d_tiles_prec(const ElGeom& g, bool fp64);   // for the tiling g.tile3d
// Tiling for a grid: the large one when it gives at least two workgroups per
// compute unit, else the shorter-column tiling of the smaller modelled time.
int el3d_choose_tiling(const ElGeom& g, bool fp64, int ncu);

// Sensitivity: per cell g = -dE/dphi * B(w,u)/E-free form, plus dot(F,u) and 2 Pi(u)
// partial sums per tile.
template <typename U, typename T>
struct ElAdjoint {
  const U* u;
  const U* w;               // may equal u
  const T* phi;             // [nphase][cells]
  T* grad;                  // [nphase][cells]
  const double* F;          // load (double, canonical layout)
  double* partial_fu;       // per tile
  double* partial_en;       // per tile
  int nphase;
  double e0, emin, p;
  double ep[kMaxPhase + 1];   // solid phases, then the void
};
template <typename U, typename T>
int launch_el2d_adjoint(const ElGeom& g, const ElAdjoint<U, T>& a, hipStream_t s);
template <typename U, typename T>
int launch_el3d_adjoint(const ElGeom& g, const ElAdjoint<U, T>& a, hipStream_t s);
// workgroups of the 3D sensitivity launch (one partial-sum slot each), the larger
// of the two state precisions
int el3d_adjoint_tiles(const ElGeom& g);

// ---------------------------------------------------------------- heat (2D batch)
struct HeatDesign {
  int nx, ny;
  long off;                 // first cell of this design in the concatenated arrays
  int tile0, ntile;         // tile range of this design in the work list
  int dir_off;              // Dirichlet side tables: [ny] left, [ny] right, [nx] bottom, [nx] top
  int pad;
  double h;
  double fsrc;              // uniform source per cell (q h^2) when the dense rhs is absent
};

struct HeatTile {
  int design, i0, j0, pad;
};

template <typename T>
struct HeatSweep {
  const T* uin;
  T* uout;
  T* v;
  T* vout;                  // multi-sweep kernel: velocity output (see ElSweep)
  const T* k;
  const T* b;               // dense rhs or nullptr (uniform source)
  const HeatDesign* des;
  const HeatTile* tiles;
  const uint8_t* dir;       // Dirichlet side tables
  const SolveState* st;     // per design
  const int* all_done;
  double* partial;          // per tile
  float* b32;               // refine: receives float(r)
  int ntile;
};
template <typename T, int MODE>
void launch_heat2d(const HeatSweep<T>& a, hipStream_t s);
// K sweeps per launch on 64x32 windows; the work list holds the inner
// (64-2K) x (32-2K) blocks.  Bit-identical to K one-sweep launches.
template <typename T, int K, bool CHECK>
void launch_heat2d_tb(const HeatSweep<T>& a, hipStream_t s);

template <typename U, typename T>
struct HeatAdjoint {
  const U* u;
  const U* w;
  const T* phi;
  T* grad;
  const double* F;          // dense source (double) per cell, or nullptr (uniform)
  const HeatDesign* des;
  const HeatTile* tiles;
  const uint8_t* dir;
  double* partial_fu;
  double* partial_en;
  double e0, emin, p;
  int ntile;
};
template <typename U, typename T>
void launch_heat2d_adjoint(const HeatAdjoint<U, T>& a, hipStream_t s);

// ---------------------------------------------------------------- generic control kernels
struct CellRange {          // one design's cell block for per-design elementwise kernels
  long off;
  long n;
  int nx, ny, nz;
  int pad;
  double h;
};

template <typename T>
void launch_material(const T* phi, T* E, double* E64, const CellRange* ranges, int ndes,
                     long max_cells, int nphase, long phase_stride, double e0, double emin,
                     double p, const double* ep, double* partial_max, int blocks_per_design,
                     hipStream_t s);

struct SetupArgs {
  SolveState* st;
  const double* partial_max;  // [ndes][blocks_per_design]
  int blocks_per_design;
  int ndes;
  const double* fnorm;        // [ndes]
  const double* h;            // [ndes]
  double m0;                  // P-wave modulus at unit modulus (heat: 1)
  int ndim;
  double theta, dt_user, tol;
  int max_iter, check_every;
  int replay;
  int adapt;
  int* ctl;                   // [0] = poll sequence, [1] = all_done
};
void launch_setup(const SetupArgs& a, hipStream_t s);

struct FinalizeArgs {
  SolveState* st;
  const double* partial;      // per tile sums
  const int* tile0;           // [ndes+1] tile ranges (prefix), or nullptr: one design, ntile tiles
  int ntile;
  int ndes;
  const long* ncell;          // [ndes]
  int* ctl;                   // [0] poll sequence, [1] all done
  PollRecord* ring;           // host-mapped ring
  int mode;                   // 0: check after the block's sweeps; 1: check before them (refinement)
  double div_factor;
  const double* prq;          // adaptive damping: [ndes][rq_blocks][3] sums of u.u, u.F, u.r
  int rq_blocks;
};

// Per-design sums of u.u, u.F and u.r over the state (FP64), for the Rayleigh
// quotient of the adaptive damping.  F: dense load (double) or nullptr (uniform
// source of the range).
template <typename U, typename R>
void launch_rq(const U* u, const R* r, const double* F, const StateRange* ranges, int ndes, int bpd,
               double* prq, hipStream_t s);
void launch_finalize(const FinalizeArgs& a, hipStream_t s);
// Adaptive damping from the sums in prq, applied to every unfinished design
// before a solve's first sweep.
void launch_adapt(SolveState* st, const double* prq, int rq_blocks, int ndes, hipStream_t s);

template <typename T>
void launch_fill(T* p, long n, T value, hipStream_t s);
// u += d, d = 0 (refinement: fold the FP32 correction into the double state);
// skipped once every design is done.
void launch_fold(double* u, float* d, long n, const int* all_done, hipStream_t s);

// ---------------------------------------------------------------- phase update
// One phase of one design: normalised sensitivity step, Allen-Cahn step into
// `work` (double), bracketed search of the volume shift, clamped apply.
template <typename T>
struct PhaseArgs {
  T* phi;                   // phase m of the design (in/out)
  const T* g;               // sensitivity of phase m
  double* used;             // sum of the phases updated before this one (upper bound
                            // 1 - used), or nullptr (bound 1)
  double* used_out;         // apply: receives used + the new phase, or nullptr
  double* work;             // phi'' of this design (double)
  double* partial;          // per block scratch, >= nblocks * 64
  double* scal;             // [0] gmax [1] lo [2] hi [3] s [4] mean phi [5] target sum
                            // [6] sum phi [7] sum phi over the void region
  int nx, ny, nz;           // cells (nz = 1 in 2D)
  int ndim;
  long n;
  double h, alpha, gamma, dt_ac, target;
  int nblocks;
  // regions (nullptr: every cell is a design cell)
  const uint8_t* region;    // PETTO_REGION_* per cell of this design
  int first;                // this is phase 0 (passive-solid cells hold it at 1)
};
template <typename T> void launch_phase_gmax(const PhaseArgs<T>& a, hipStream_t s);
template <typename T> void launch_phase_step(const PhaseArgs<T>& a, hipStream_t s);
template <typename T> void launch_phase_pass(const PhaseArgs<T>& a, hipStream_t s);
template <typename T> void launch_phase_apply(const PhaseArgs<T>& a, hipStream_t s);
int phase_blocks(long n);

// The paper's penalty update and Cahn-Hilliard step for every stored phase of
// one design, in six launches whatever the phase count.
template <typename T>
struct PenaltyArgs {
  T* phi;                   // phase 0 of the design (in/out); phase m at + m * pstride
  const T* g;               // sensitivity, same layout
  long pstride;             // elements between phases (the context's cell count)
  int nphase;
  double* p1;               // phi' of phase m at + m * mstride (double)
  double* mu;               // chemical potential of phase m at + m * mstride (double)
  long mstride;
  double* partial;          // per block scratch, >= 3 * nphase * nblocks
  double* scal;             // phase m: scal + 8 m ([0] max|g| [1] volume-penalty term
                            // [3] its negative [4] new mean [6] sum phi [7] sum over the void region)
  int nx, ny, nz, ndim;     // cells (nz = 1 in 2D)
  long n;
  double h, alpha, gamma, alpha_v, alpha_1, dt_ch, mobility, alpha_b;
  double vol_frac[kMaxPhase];
  const uint8_t* region;    // PETTO_REGION_* per cell, or nullptr
  int nblocks;
};
template <typename T> void launch_penalty_update(const PenaltyArgs<T>& a, hipStream_t s);

// out[2d] = sum of pfu over design d's tiles, out[2d+1] = the same for pen.
void launch_dot_finalize(const double* pfu, const double* pen, const int* tile0, int ntile, int ndes,
                         double* out, hipStream_t s);

}  // namespace petto
