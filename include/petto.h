/*
 * petto.h -- C ABI of the MI355X (gfx950) pseudo-transient topology-optimisation path.
 *
 * The operations follow the PDE-constrained statement of Section 2.1 (Eq. 2.1):
 * a design phi determines a state u with R(u, phi) = 0 (linear elasticity,
 * Eqs. 3.6, 3.9, 3.10, or steady heat conduction, Eq. 2.2), an objective
 * (compliance, Eq. 2.7 / Eq. 3.7) with its sensitivity (Section 2.3), and a
 * constrained design update (Sections 2.4 and 3.1, Eqs. 2.15, 3.2, 3.3), chained as
 * one optimisation loop of the workflow in Fig. 4.
 *
 * Conventions for every entry point
 *  - Pointers named "device" address GPU memory owned by the caller; the library
 *    never frees, reallocates or keeps them beyond the call, except that cached
 *    launch graphs record their addresses (passing other buffers re-records).
 *  - Pointers named "host" address CPU memory; they are read (or written) only
 *    during the call.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls are ordered on it.
 *  - A negative status is an error: outputs are undefined, inputs unchanged, and
 *    petto_last_error() returns a message.  Argument checks run before any GPU
 *    work, so they are safe without a GPU.  Nothing throws across the ABI.
 *  - Floating-point buffers are in the context precision (float for PETTO_FP32,
 *    double for PETTO_FP64) unless stated otherwise.  All norms, volume sums,
 *    compliance values and the volume-multiplier search run in double.
 *
 * Canonical layouts (x fastest, row-major)
 *  - Elastic state-like arrays (u, v, loads, Dirichlet mask): component-major and
 *    padded, [d][nz+1][ny+1][nx+1] (2D: [d][ny+1][nx+1]).  Component a lives on the
 *    faces normal to axis a: its index along a runs 0..n_a, along any other axis b
 *    0..n_b-1; the slot with index n_b on a foreign axis is padding (kept zero).
 *  - Cell arrays (phi, grad_phi, temperature): [nphase][nz][ny][nx].
 *  - Heat Dirichlet faces: one byte per cell, bit 2a = face on the low side of
 *    axis a, bit 2a+1 = face on the high side.
 *  - A batch of designs (heat) is the concatenation of the designs' arrays; see
 *    petto_field_offset().
 */
#ifndef PETTO_H
#define PETTO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct petto_ctx petto_ctx;

typedef enum {
  PETTO_OK = 0,
  PETTO_NOT_CONVERGED = 1,   /* max_iter reached; outputs valid */
  PETTO_ERR_INVALID = -1,    /* bad argument */
  PETTO_ERR_HIP = -2,        /* HIP runtime failure */
  PETTO_ERR_DIVERGED = -3,   /* residual non-finite or grew by 1e4 over the first check */
  PETTO_ERR_OOM = -4,        /* device allocation failed */
  PETTO_ERR_UNSUPPORTED = -5 /* valid but not implemented combination */
} petto_status;

enum { PETTO_ELASTIC = 0, PETTO_HEAT = 1 };
enum { PETTO_FP32 = 0, PETTO_FP64 = 1 };
enum { PETTO_SIDE_FREE = 0, PETTO_SIDE_CLAMPED = 1, PETTO_SIDE_ROLLER = 2 };
enum { PETTO_FIELD_STATE = 0, PETTO_FIELD_CELL = 1 };
/* Cell roles.  VOID: every solid phase held at 0 by the Allen-Cahn update's bounds,
 * and the J_b penalty of the penalty model (weight alpha_b).  SOLID: phase 0 held
 * at 1 (the other phases at 0) after either update. */
enum { PETTO_REGION_DESIGN = 0, PETTO_REGION_VOID = 1, PETTO_REGION_SOLID = 2 };

#define PETTO_MAX_PHASES 6

/* One design problem (Section 2.1).  Material law: single phase uses the modified
 * SIMP form  E = emin + phi^p (e0 - emin)  (heat: k, same form); nphase = N in
 * 2..PETTO_MAX_PHASES stores N solid phases and
 * E = sum_m e_phase[m] phi_m^p + e_phase[N] (1 - sum_m phi_m)^p (Eq. 3.8 with an
 * implicit void phase).  Fractions enter the laws clamped to [0, 1].  Elastic 2D uses the Lame parameters of
 * Eq. 3.10 as printed (plane strain).
 *  side[6]: boundary type of the -x,+x,-y,+y,-z,+z sides.  CLAMPED fixes both
 *           components (normal unknown zero, tangential reflected); ROLLER fixes the
 *           normal unknown only; FREE is traction free.  Heat ignores side[].
 *  fixed:   host, may be NULL.  Elastic: one byte per unknown in the canonical
 *           layout, nonzero = Dirichlet (held at zero).  It must include the normal
 *           unknowns of every CLAMPED/ROLLER side.  Heat: per-cell face bits (above);
 *           a heat design needs at least one Dirichlet face.
 *  load:    host, may be NULL.  Force per unknown in force units (double), canonical
 *           layout (heat: per-cell source already multiplied by h^d).  Heat with
 *           load == NULL uses the uniform source density q.  Elastic needs a load. */
typedef struct {
  int32_t physics;          /* PETTO_ELASTIC or PETTO_HEAT */
  int32_t ndim;             /* 2 or 3 (heat: 2) */
  int32_t n[3];             /* cells along x, y, z (n[2] ignored in 2D) */
  double h;                 /* grid spacing */
  double e0, emin, nu, p;   /* SIMP law; nu ignored for heat */
  int32_t nphase;           /* 1, or 2..PETTO_MAX_PHASES (elastic only) */
  double e_phase[PETTO_MAX_PHASES + 1];  /* nphase >= 2: the solid phases, then the void */
  int32_t side[6];
  const uint8_t *fixed;
  const double *load;
  double q;
  const uint8_t *region;    /* host, one byte per cell ([nz][ny][nx]) or NULL: PETTO_REGION_*
                               (the void region of Section 3.4 and passive solid cells) */
} petto_problem;

/* Pseudo-transient relaxation controls (Section 2.2, Eqs. 2.5-2.6 / 3.12).
 *  sweep:  v <- (theta v + dt R(u)) / (theta + dt),  u <- u + dt v,  R = (F - K u) / h^d.
 *  theta = 0 is plain PT (Eq. 2.4 / 3.11).  dt <= 0 selects h sqrt(theta / (2 d M_max))
 *  (theta > 0) or h^2 / (2 d M_max) (theta = 0), M_max the largest P-wave modulus
 *  lam + 2 mu over the cells (heat: largest conductivity).
 *  Stop rule: every check_every-th sweep, rho = ||F - K u||_2 / ||F||_2 of the state
 *  that sweep starts from; stop after that sweep once rho <= tol.
 *  refine (FP32 contexts): the state u is double and the sweeps run in FP32 on a
 *  correction d with right-hand side r64 = F - K u (double, rounded to float); at
 *  every check the correction is folded into u (u += d, d = 0) and r64 is
 *  recomputed in double, so the stop rule sees the double residual of u.  The
 *  velocity carries over, so in exact arithmetic this is the same iteration.
 *  use_graph: replay captured blocks of check_every sweeps instead of launching
 *  each sweep from the host.  replay_iters > 0: run exactly that many sweeps (a
 *  multiple of check_every), ignoring tol.
 *  adapt: choose the damping from the starting state u before the first sweep
 *  (a state of zeros keeps theta_given) and re-choose it from the state at every
 *  check block boundary: theta = max(theta_given, 1 / (4 lam)) with the Rayleigh
 *  quotient lam = u.K u / (h^d u.u), which critically damps the mode of the
 *  current state (needs dt <= 0: the step follows theta).  The velocity carries
 *  over. */
typedef struct {
  double theta;
  double dt;
  double tol;
  int32_t max_iter;
  int32_t check_every;      /* even, >= 2 */
  int32_t refine;
  int32_t use_graph;
  int32_t replay_iters;
  int32_t adapt;
  int32_t n_pt;             /* > 0: after the damped-wave sweeps, n_pt plain PT sweeps
                               (theta = 0, even count, no stop rule): the paper's
                               hybrid schedule (Section 3, n_APT + n_PT per loop) */
  double dt_pt;             /* PT step of that stage; <= 0: h^2 / (2 d M_max) */
} petto_apt_params;

enum { PETTO_UPDATE_ALLEN_CAHN = 0, PETTO_UPDATE_PENALTY_CH = 1 };

/* Design update controls (Sections 2.4, 3.1).
 * model PETTO_UPDATE_ALLEN_CAHN:   phi' = phi - alpha_h g / max|g|
 * (Eq. 3.2 step), phi'' = phi' - dt_ac (w'(phi') - gamma lap phi') with
 * w = sin^2(pi phi)/64 (Eq. 2.15) and mirror boundaries, then
 * phi = clamp(phi'' + s, 0, ub) with s such that mean(phi) = vol_frac (ub = 1 for
 * the first phase, 1 minus the already updated phases for the later ones).
 * dt_ac <= 0 selects 0.9 min(h^2 / (4 d gamma), 32 / pi^2).  bisect_passes <= 0 selects the default
 * (9 passes of a 64-way bracket split, bracket width <= 2^-54 of the start).
 * model PETTO_UPDATE_PENALTY_CH (the paper's own update, Eq. 2.13 with the
 * normalised sensitivity of Section 3.1, then one explicit step of Eq. 2.14):
 *   phi' = phi - alpha_h g / max|g| - alpha_v dJ_v/dphi - alpha_1 dJ_1/dphi,
 *   dJ_v/dphi = 2 (h^d sum phi - vol_frac N h^d) h^d,  dJ_1/dphi = 2 (sum_m phi_m - 1) h^d,
 *   phi = phi' + dt_ch D lap(w'(phi') - gamma lap phi'), mirror boundaries,
 * every phase from the same old design; no clamp and no projection (the material
 * laws evaluate fractions clamped to [0, 1]).  info.shift receives the uniform
 * volume-penalty term -alpha_v dJ_v/dphi. */
typedef struct {
  double alpha_h;
  double gamma;
  double dt_ac;
  double vol_frac[PETTO_MAX_PHASES];
  int32_t bisect_passes;
  int32_t model;            /* PETTO_UPDATE_ALLEN_CAHN (above) or PETTO_UPDATE_PENALTY_CH */
  double alpha_v;           /* penalty model: volume-penalty weight (paper: 1e5) */
  double alpha_1;           /* penalty model: partition-of-unity weight (0 with an implicit void) */
  double dt_ch;             /* penalty model: Cahn-Hilliard step; <= 0: 500 h^4 capped at 0.9
                               of the step's stability limit 2 / (D lam (pi^2/32 + gamma lam)),
                               lam = 4 d / h^2 (the cap binds in 3D) */
  double mobility;          /* penalty model: D of Eq. 2.14; <= 0: 1 */
  double alpha_b;           /* penalty model: void-region weight, J_b = (int_{Omega_b} phi - 0)^2 */
} petto_phase_params;

typedef struct {
  int32_t iters;            /* sweeps run (all correction solves together) */
  int32_t status;           /* petto_status of this design */
  int32_t outer;            /* refine: double-residual checks run */
  int32_t pad_;
  double rel_res;           /* rho at the last check (refine: double residual) */
  double r_pde;             /* Eq. 3.5: sqrt(sum R^2) / number of cells */
  double dt;                /* pseudo-time step at the end */
  double theta;             /* damping at the end */
} petto_solve_info;

typedef struct {
  double shift[PETTO_MAX_PHASES];   /* volume multiplier s per phase (penalty model: -alpha_v dJ_v/dphi) */
  double volume[PETTO_MAX_PHASES];  /* mean(phi) per phase after the update */
  double gmax[PETTO_MAX_PHASES];    /* max |g| per phase used for normalisation */
} petto_phase_info;

/* Create a context for nprob designs in precision prec (PETTO_FP32 / PETTO_FP64).
 * Elastic: nprob must be 1.  Heat: any nprob >= 1 (a batch, solved in shared
 * launches).  Copies the problem data (masks, loads) to the device.  *out receives
 * the context (owned by the caller; release with petto_destroy).  3D elastic
 * problems need (n[0]+1)(n[1]+1) < 2^29 (one xy layer of positions addressed by
 * 32-bit byte offsets), else PETTO_ERR_UNSUPPORTED. */
petto_status petto_create(const petto_problem *probs, int32_t nprob, int32_t prec, petto_ctx **out);

/* Release a context and everything it owns.  NULL is accepted. */
petto_status petto_destroy(petto_ctx *ctx);

/* Offset (in elements) of design iprob inside a concatenated buffer of kind field
 * (PETTO_FIELD_STATE: u/v layout; PETTO_FIELD_CELL: one phase of phi/grad) and the
 * total element count of such a buffer (iprob == nprob).  Returns (size_t)-1 on bad
 * arguments. */
size_t petto_field_offset(const petto_ctx *ctx, int32_t iprob, int32_t field);

/* Relax the state (Section 2.2) for design phi (device, cell layout), starting from
 * u (device; double when refine is set, context precision otherwise) and zero
 * velocity v (device, context precision, overwritten).  On return u holds the
 * relaxed state and info (host, nprob entries, may be NULL) the solve record.
 * Returns PETTO_OK if every design met tol, PETTO_NOT_CONVERGED if one hit max_iter,
 * PETTO_ERR_DIVERGED if one diverged.  Synchronous: returns after the GPU work,
 * except for fixed-count stages called with info == NULL while sweep timing is
 * off (replay_iters > 0, and the n_pt stage): those are only enqueued on stream,
 * so with replay_iters > 0 the call returns PETTO_OK at once (divergence is then
 * not reported; the device still stops a diverged design). */
petto_status petto_apt_solve(petto_ctx *ctx, const void *phi, void *u, void *v,
                             const petto_apt_params *params, void *stream, petto_solve_info *info);

/* Force residual r = F - K(phi) u (device; same layout and precision as u; zero on
 * Dirichlet and padding slots).  One application of the operator the sweeps use. */
petto_status petto_residual(petto_ctx *ctx, const void *phi, const void *u, void *r, void *stream);

/* Compliance and its sensitivity (Section 2.3, Eq. 2.7 / 3.7): grad_phi (device,
 * cell layout, context precision) receives dC/dphi = -dE/dphi * B_c(w, u) / E_c
 * with the cell bilinear energy form B_c (B_c(u,u) = 2 W_c), w = u when w is NULL
 * (self-adjoint compliance).  u and w are double when `state_fp64` is nonzero,
 * else context precision.  compliance (device, double[2*nprob], may be NULL)
 * receives {F.u, 2 Pi(u)} per design.  Asynchronous on stream.  The context's
 * partial-sum buffers are sized for this launch at creation; should they not
 * fit, the call returns PETTO_ERR_UNSUPPORTED before launching anything. */
petto_status petto_adjoint(petto_ctx *ctx, const void *phi, const void *u, const void *w,
                           int32_t state_fp64, void *grad_phi, double *compliance, void *stream);

/* petto_adjoint without the context's workspace, for callers that cannot
 * allocate or must not touch allocating calls (code under HIP graph capture,
 * tight serving loops): same arguments, results and error behaviour as
 * petto_adjoint (bit-identical outputs), but its partial sums live in one fixed
 * device array of the library, 2 x 65536 doubles (1 MiB) per GPU, held until
 * the process ends; the call allocates nothing.  A launch needing more than
 * 65536 partial-sum slots (one per workgroup: about 1024 x 512 cells per 10,000
 * slots in 2D, 1.4 M positions per 10,000 in 3D) returns PETTO_ERR_UNSUPPORTED
 * before any GPU work.  The array is shared by every call on a GPU and keeps
 * the last call's contents: calls that overlap on one GPU (other streams, other
 * threads) race on it and must be serialized by the caller.  The array's device
 * address is resolved at petto_create, so a context must have been created on
 * the current GPU (else PETTO_ERR_INVALID). */
petto_status petto_adjoint_noalloc(petto_ctx *ctx, const void *phi, const void *u, const void *w,
                                   int32_t state_fp64, void *grad_phi, double *compliance, void *stream);

/* Design update in place (normalised sensitivity step, Allen-Cahn step, volume
 * projection).  phi (device) is overwritten; grad_phi (device) is read.  info (host,
 * nprob entries, may be NULL): when given the call waits for the GPU work. */
petto_status petto_phase_update(petto_ctx *ctx, void *phi, const void *grad_phi,
                                const petto_phase_params *params, void *stream,
                                petto_phase_info *info);

/* One optimisation loop of Fig. 4: petto_apt_solve, petto_adjoint (w = u), then
 * petto_phase_update.  grad_phi (device) receives the sensitivity used;
 * compliance (device double[2*nprob], may be NULL) as in petto_adjoint.  With a
 * fixed sweep count and sinfo == pinfo == NULL the whole loop is only enqueued on
 * stream (no host wait), so successive calls run back to back on the GPU. */
petto_status petto_step(petto_ctx *ctx, void *phi, void *u, void *v, void *grad_phi,
                        double *compliance, const petto_apt_params *ap,
                        const petto_phase_params *pp, void *stream,
                        petto_solve_info *sinfo, petto_phase_info *pinfo);

/* Mean duration in milliseconds of the sweep kernels of the last petto_apt_solve
 * (timed with HIP events on the solve stream around whole launches of sweep
 * blocks, four blocks per launch when graphs are used), and the number of sweeps
 * those blocks held (for a solve stopped by tol, counting the blocks of its last
 * launch).  Returns 0 when nothing was timed. */
double petto_last_sweep_ms(const petto_ctx *ctx, int64_t *sweeps);

/* Enable (1) or disable (0) the sweep timing above (off by default). */
petto_status petto_set_timing(petto_ctx *ctx, int32_t on);

/* Sweeps per launch of the 2D relaxations (elastic and heat).  k in {2, 4, 5, 8, 10}
 * (FP64: {2, 4, 5}): each launch stages an LDS window of the grid and runs k sweeps
 * on it (results bit-identical to one sweep per launch); k = 1: one sweep per
 * launch; k = 0 (the default, FP32 and FP64): the first solve times every
 * candidate that divides its check blocks on workspace buffers and keeps the
 * fastest; the choice is cached for the process per (physics, dimension,
 * precision, check interval, compute units, grid sizes), so later contexts of
 * the same shape reuse it.  A block of check_every sweeps uses k only when
 * check_every is a multiple of 2k, else one sweep per launch.  3D contexts
 * stream along z with one sweep per launch (tiling: petto_set_tile3d). */
petto_status petto_set_blocking(petto_ctx *ctx, int32_t k);

/* The sweeps per launch in use (0: not timed yet). */
int32_t petto_blocking(const petto_ctx *ctx);

/* Tiling of the 3D elastic sweeps (streamed along z, Eqs. 3.6 and 3.12 in 3D):
 * t = 1: columns of 64 x 8 positions through 16 layers (FP64: 64 x 4 through 8),
 * the fewest halo bytes; t = 2: columns of 64 x 4 positions through 4 layers and t = 3:
 * through 2 layers, more workgroups for small grids; t = 0 (the default): the first
 * solve times the three on workspace buffers and keeps the fastest (cached per
 * shape like the sweeps per launch; until then a model of resident workgroups
 * picks one).  Results are bit-identical for all tilings except the order of the
 * FP64 residual-norm sum.  Errors: PETTO_ERR_INVALID for other values or a context
 * that is not 3D elastic.  Cached launch graphs are dropped. */
petto_status petto_set_tile3d(petto_ctx *ctx, int32_t t);

/* The 3D tiling in use (1, 2 or 3; 0 for a NULL context). */
int32_t petto_tile3d(const petto_ctx *ctx);

/* Time the context's dominant sweep kernel (the relaxation launch of Eq. 3.12 /
 * the heat analogue, with the current sweeps per launch and tiling): `launches`
 * (2..100000, rounded up to even) back-to-back launches, without checks, on
 * workspace buffers (zero state; the caller's buffers are untouched) with the
 * step coefficients of the last solve, bracketed by two HIP events on `stream`.
 * Writes the mean milliseconds per launch and the sweeps each launch performs.
 * Blocks until done.  FP32 contexts only (PETTO_ERR_UNSUPPORTED otherwise). */
petto_status petto_time_sweeps(petto_ctx *ctx, int32_t launches, void *stream, double *ms_per_launch,
                               int32_t *sweeps_per_launch);

/* Message of the last failure on the calling thread ("" if none). */
const char *petto_last_error(void);

/* Library version string. */
const char *petto_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PETTO_H */
