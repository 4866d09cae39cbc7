/*
 * lbm.h -- C ABI of the MI355X (gfx950) wall-modeled LBM-LES library.
 *
 * The library advances the homogenized lattice Boltzmann update of
 * Kummerlaender et al., arXiv 2506.21804, Sec. 2.2, Eq. (6), in its BGK form
 * with the Smagorinsky effective relaxation time (Sec. 2.1, Eqs. (3)-(5);
 * Sec. 2.2, Eq. (14)), the homogenized velocity of Eq. (12) and Guo body
 * forcing, on a D3Q19 (the paper's stencil, Sec. 2.2) or D3Q27 lattice,
 * with halfway bounce-back on a voxel geometry and the Spalding wall model
 * of Sec. 2.2.1 (Eqs. (15)-(17); sigma = 0 and the modeled velocity as the
 * solid velocity in wall cells).  Populations live in one in-place buffer
 * (AA pattern) in structure-of-arrays order as deviations from the rest
 * weights, g_i = f_i - w_i, stored in FP64, FP32 or IEEE binary16.
 *
 * Conventions shared by every entry point:
 *  - cell index c = x + nx*(y + ny*z); N = nx*ny*nz, 1 <= N < 2^31;
 *  - scalar fields are [N], vector fields [3][N] (component-major),
 *    population fields [q][N];
 *  - "compute type" is double for LBM_F64 storage and float otherwise;
 *  - device pointers are HIP device memory owned by the caller; the library
 *    never allocates or frees device memory, and keeps no pointer to host
 *    inputs after a call returns;
 *  - all device work is enqueued on params.stream (NULL = the null stream);
 *    calls marked "async" return before the work finishes;
 *  - every function returns LBM_OK or a negative code and stores a message
 *    readable with lbm_last_error(); a failed argument check has no side
 *    effects.  Faults detected inside kernels (a non-finite density, a
 *    wall-function Newton failure) are reported by the next synchronising
 *    call (lbm_sync, lbm_diagnostics, lbm_objective, lbm_gradient).
 *  - a context is not thread-safe; use one per host thread.
 */
#ifndef LBM_MI355X_H
#define LBM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* invalid argument */
  LBM_EHIP = -2,       /* a HIP runtime call or kernel launch failed */
  LBM_ENONFINITE = -3, /* a cell density became non-finite or non-positive */
  LBM_ENEWTON = -4,    /* the wall-function Newton solve failed */
  LBM_ESIZE = -5       /* workspace or buffer too small, or domain too large */
};

enum { LBM_D3Q19 = 19, LBM_D3Q27 = 27 };
enum { LBM_F64 = 0, LBM_F32DEV = 1, LBM_F16DEV = 2 };
/* Collision model of the bulk (sigma = 1) update, Sec. 2.2:
 *  LBM_BGK: second-order equilibrium, all of f - f^eq relaxed (Eq. (6));
 *  LBM_RR3: recursive regularized, third order: third-order equilibrium
 *    (Eq. (11)) and f^(1) rebuilt from its Hermite coefficients of order 1
 *    to 3 (Eqs. (8), (9)), the third by the recursion u_a Pi_bc + u_b Pi_ac
 *    + u_c Pi_ab; third-order terms projected on the Hermite components the
 *    lattice carries.  Wall cells and the initial state then use the
 *    third-order equilibrium as well.  The adjoint supports both models. */
enum { LBM_BGK = 0, LBM_RR3 = 1 };

typedef struct {
  int lattice;        /* LBM_D3Q19 or LBM_D3Q27 */
  int nx, ny, nz;     /* domain size in cells */
  int periodic[3];    /* per axis; outside a non-periodic axis is solid */
  int storage;        /* LBM_F64 | LBM_F32DEV | LBM_F16DEV */
  double tau0;        /* molecular relaxation time, nu = (tau0 - 1/2)/3, > 1/2 */
  double cs_smag;     /* Smagorinsky constant C_S (filter width = 1 cell), >= 0 */
  double force[3];    /* body force per unit volume, lattice units (Guo) */
  int wall_model;     /* 0: bounce-back only; 1: Spalding wall model on wall cells */
  double kappa, E;    /* Spalding constants (0.41, 9.0 for a smooth wall) */
  int fringe_len;     /* urban open boundary: fringe over the last planes in x (0 = off) */
  double u_ref, z0;   /* log-law inflow u_ref ln(1 + z_c/z0)/ln(1 + z_top/z0) */
  int lid;            /* 1: the top plane z = nz-1 holds the inflow equilibrium */
  int collision;      /* LBM_BGK or LBM_RR3 */
  double fd_weight;   /* 1 - sigma of Eq. (7), in [0, 1], above 0 only with LBM_RR3:
                       * weight of the finite-difference strain (Eq. (10)) taken
                       * from central differences of the step's velocity field;
                       * wall cells then use the full finite-difference strain
                       * with its wall-normal shear replaced by the wall law's.
                       * 0 = purely local. */
  int open_x;         /* 1: open x faces (Sec. 2.2.2, Sec. 3.2): regularized local
                       * velocity inlet on the plane x = 0 imposing (u_in(z), 0, 0),
                       * the log-law profile above; fixed local pressure outlet on
                       * x = nx-1 imposing rho_out with zero tangential velocity.
                       * Each such fluid cell that is not a lid cell rebuilds its
                       * pre-collision populations, then collides as a bulk cell:
                       * inlet cells as f^eq(rho, u) plus the regularized
                       * non-equilibrium (the unknown populations, those entering
                       * through the face, take the non-equilibrium of their
                       * opposites); outlet cells as f^eq(rho_out, u) with the
                       * normal velocity from the known populations.  Needs a
                       * non-periodic x axis, nx >= 3, fringe_len <= nx - 2 (the
                       * outlet plane is left out of the fringe), no force, no
                       * hybrid (fd_weight 0), z0 > 0; these cells are never
                       * wall-modeled.  0 = off. */
  double rho_out;     /* outlet density, > 0 (open_x only) */
  int slip;           /* full-slip box faces (Sec. 3.2, the outer walls of the street
                       * canyon): bit 2a the low face of axis a (x 0, y 1, z 2), bit
                       * 2a+1 the high face; only on non-periodic axes, not on open
                       * x faces, not on the top face with a lid.  A population
                       * that crosses such faces is reflected specularly: it
                       * arrives at the cell one step along its direction with
                       * the crossed components set to zero, with those velocity
                       * components negated (halfway bounce-back where that cell
                       * is solid).  These links are not walls of the wall model;
                       * the voxel wall distance mirrors the geometry across them.
                       * 0 = none (outside a non-periodic axis is a no-slip wall). */
  int cs_field;       /* 1 reserves workspace for a per-cell Smagorinsky constant
                       * (lbm_set_smagorinsky); 0 = the scalar cs_smag only */
  void *stream;       /* hipStream_t for all device work (NULL = null stream) */
} lbm_params;

/* Device bytes the caller must provide to lbm_init for these parameters and
 * this host mask (uint8 [N], 1 = fluid; NULL = all fluid).  Returns 0 on
 * invalid parameters.  porous != 0 reserves room for a porosity field. */
size_t lbm_workspace_bytes(const lbm_params *p, const uint8_t *mask, int porous);

/* Creates a context, builds the cell flags and wall-cell records on the host
 * (wall cells: fluid cells with a solid link; normal from the sum of solid
 * links; reference cell one step along the best-aligned lattice direction),
 * uploads them, and writes f^0 = f^eq(rho0, u0) (Sec. 2.2 second-order
 * equilibrium).  Synchronises the stream before returning.
 *   mask      host uint8 [N], 1 = fluid, 0 = solid; NULL = all fluid
 *   wall_dist host double [N], distance from each cell centre to the wall,
 *             read at wall cells and their reference cells only; NULL with
 *             wall_model = 1 makes the library compute the voxel distance
 *             (nearest solid unit cube within two cells, outside = solid)
 *   porosity  host double [N] in [0,1] (1 = fluid; Eq. (12) read with
 *             d = 1 - porosity); NULL = 1 everywhere
 *   rho0, u0  DEVICE double [N] and [3][N] initial fields; NULL = 1 and 0
 *   workspace device memory of at least lbm_workspace_bytes(p, mask,
 *             porosity != NULL) bytes, caller-owned, 256-byte aligned,
 *             not touched by the caller while the context lives. */
int lbm_init(lbm_ctx **out, const lbm_params *p, const uint8_t *mask, const double *wall_dist,
             const double *porosity, const double *rho0, const double *u0, void *workspace,
             size_t workspace_bytes);

/* Advances n >= 0 time steps (async).  Each step: the wall records (u_tau by
 * Newton in FP64 from the Spalding law at each wall cell's reference cell)
 * and the wall reconstruction, then the fused collide-and-stream of all other
 * fluid cells. */
int lbm_step(lbm_ctx *ctx, int n);

/* Density and velocity u = (j + F/2)/rho of the current state into device
 * buffers of the compute type, rho [N] and u [3][N]; solid cells give 0
 * (async). */
int lbm_moments(lbm_ctx *ctx, void *rho, void *u);

/* Total mass and momentum over fluid cells of the current state, summed in
 * FP64 in a fixed order (deterministic): out = {M, Px, Py, Pz}.  Synchronises
 * and reports kernel-side faults. */
int lbm_diagnostics(lbm_ctx *ctx, double out[4]);

/* lbm_diagnostics for callers that cannot allocate device memory or must not
 * depend on the workspace's reduction region (code under stream capture,
 * tight serving loops): the same sums, computed by the same kernels in the
 * same order (bit-identical results), with the reduction partials and sums
 * held in a static device array of the library (1024 x 8 + 8 doubles, 64 KiB,
 * one copy per GPU, kept until the process ends; its address is looked up
 * once per device by lbm_init).  Allocates nothing.  The array is shared by
 * every call on one GPU and holds the last call's values: calls that overlap
 * on one GPU (two streams, two threads) race.  Any domain lbm_init accepts
 * fits (the reduction never uses more than 1024 partials); a reduction that
 * would need more gives LBM_ESIZE.  Synchronises and reports kernel-side
 * faults like lbm_diagnostics. */
int lbm_diagnostics_noalloc(lbm_ctx *ctx, double out[4]);

/* Waits for the stream and reports kernel-side faults. */
int lbm_sync(lbm_ctx *ctx);

/* Shape of a context: out = {q, nx, ny, nz, storage}. */
int lbm_shape(const lbm_ctx *ctx, int out[5]);

/* Number of time steps taken since lbm_init (or the loaded state). */
long long lbm_steps_done(const lbm_ctx *ctx);

/* Current populations f_i = w_i + g_i in natural order [q][N] of the compute
 * type (device, async); solid cells give 0. */
int lbm_get_populations(lbm_ctx *ctx, void *f);
/* Replaces the state by the populations f [q][N] of the compute type
 * (device, async); values at solid cells are ignored. */
int lbm_set_populations(lbm_ctx *ctx, const void *f);

/* Snapshot of the state (populations in their in-memory layout plus the step
 * counter) into / from caller device memory of lbm_state_bytes() bytes
 * (async D2D copies; load reads the step counter synchronously). */
size_t lbm_state_bytes(const lbm_ctx *ctx);
int lbm_save_state(lbm_ctx *ctx, void *dst);
int lbm_load_state(lbm_ctx *ctx, const void *src);

/* Terminal objective of the porosity-gradient problem:
 * J = c_s^2 (<rho>_{x=planes[0]} - <rho>_{x=planes[1]}) + <rho |u|^2 / 2>,
 * means over the fluid cells of each plane / of the domain, u the Guo
 * velocity.  Synchronises; *J in FP64. */
int lbm_objective(lbm_ctx *ctx, const int planes[2], double *J);

/* Discrete adjoint.  An adjoint field lambda is caller device memory of
 * lbm_adjoint_bytes(), 8-byte aligned, in the library's own form: per fluid
 * cell one FP64 common mode, plus q deviations in the compute type (FP64
 * for FP64 storage, FP32 otherwise) in the in-memory AA order of the current
 * step parity.  Its values are read and written in natural order through
 * lbm_adjoint_to_natural / _from_natural.  The common mode is handled in
 * FP64 and the deviations pass through the collision's vector-Jacobian
 * product in the compute precision; grad_phi is FP64.  With the hybrid
 * collision (fd_weight > 0, Eqs. (7), (10)) the buffer also holds the
 * adjoint of each cell's finite-difference strain (six values per cell in
 * the compute type, scratch of the reverse step), and the reverse step
 * carries it back through the strain's central and one-sided differences
 * to the neighbours' velocities and populations.  Misaligned buffers give
 * LBM_EINVAL.
 *  lbm_adjoint_seed: lambda = dJ/df of the current state (async).
 *  lbm_adjoint_step: given lambda = dJ/df^{n+1} and the state f^n currently
 *    held by the context (step counter n), overwrites lambda with dJ/df^n
 *    and adds dJ/dphi contributions of step n to grad_phi [N] (double);
 *    decrements nothing (the caller restores f^{n-1} itself).  With the
 *    hybrid collision it first rebuilds the workspace's velocity field from
 *    f^n (the next forward step rebuilds it again).  Async.
 *  lbm_adjoint_to_natural / _from_natural: convert lambda between its
 *    in-memory form at the current parity and natural [q][N] order (FP64
 *    values; solid cells read as 0). */
size_t lbm_adjoint_bytes(const lbm_ctx *ctx);
int lbm_adjoint_seed(lbm_ctx *ctx, const int planes[2], void *lambda);
int lbm_adjoint_step(lbm_ctx *ctx, void *lambda, void *grad_phi);
int lbm_adjoint_to_natural(lbm_ctx *ctx, const void *lambda, void *natural);
int lbm_adjoint_from_natural(lbm_ctx *ctx, const void *natural, void *lambda);

/* Gradient dJ/dphi after T steps from the current state (which becomes step
 * 0 of the sweep), by a binomial checkpointing reverse sweep (Griewank-
 * Walther): snapshots is caller device memory for nsnap >= 1 states of
 * lbm_state_bytes() each, lambda of lbm_adjoint_bytes(), grad_phi [N]
 * doubles (overwritten).  The schedule's first descent doubles as the
 * forward sweep: it stores checkpoints on its way to step T-1, takes one
 * more step for the objective and the seed, and re-advances from the last
 * checkpoint to T-1.  *J receives the objective at step T and *nforward the
 * forward steps taken (lbm_revolve_cost(T, nsnap) + 1 + that re-advance; T
 * exactly when nsnap > T).  On return the context holds the state of step 0
 * again.  Synchronises. */
int lbm_gradient(lbm_ctx *ctx, int T, const int planes[2], void *snapshots, int nsnap, void *lambda,
                 void *grad_phi, double *J, long long *nforward);

/* The same sweep for the time-averaged objective J = (1/T) sum_{t=1..T} j(f_t),
 * with j the terminal objective above: the forward values are summed on the
 * schedule's first descent, and each reverse step t >= 1 adds j'(f_t)/T to
 * lambda inside the adjoint kernel.  *J receives the average.  Same
 * arguments, conditions and synchronisation as lbm_gradient. */
int lbm_gradient_mean(lbm_ctx *ctx, int T, const int planes[2], void *snapshots, int nsnap, void *lambda,
                      void *grad_phi, double *J, long long *nforward);

/* The forward-step count of the optimal binomial schedule for T steps and
 * nsnap snapshot slots (host only; the starting state occupies one slot). */
long long lbm_revolve_cost(int T, int nsnap);

/* Per-cell Smagorinsky constant (Sec. 2.3: the dynamics take C_S from the
 * cell).  cs: DEVICE double [N], C_S >= 0 and finite at every cell (solid
 * cells included; their value is unused), copied into the workspace in the
 * compute type (FP64 for FP64 storage, FP32 otherwise); NULL returns to the
 * scalar lbm_params.cs_smag.  Needs lbm_params.cs_field = 1 at lbm_init
 * (LBM_EINVAL otherwise).  From the next step on, the bulk collision takes
 * tau_eff with the cell's own C_S, and each wall record's G and tau_b the
 * wall cell's.  A rejected field (negative, NaN or infinite entry) gives
 * LBM_EINVAL and leaves the previous C_S in force.  Synchronises. */
int lbm_set_smagorinsky(lbm_ctx *ctx, const double *cs);

/* Gradients with respect to the per-cell Smagorinsky constant as well.
 *  lbm_adjoint_step_cs: lbm_adjoint_step that also adds dJ/dC_S of step n
 *    to grad_cs [N] (double, device).  The derivative is taken at the C_S in
 *    force: the field, or the scalar cs_smag at every cell.
 *  lbm_gradient_cs: the checkpointed sweep of lbm_gradient (mean = 0) or
 *    lbm_gradient_mean (mean = 1) with grad_cs [N] overwritten by dJ/dC_S
 *    next to grad_phi.  Same conditions and synchronisation; solid cells
 *    read 0. */
int lbm_adjoint_step_cs(lbm_ctx *ctx, void *lambda, void *grad_phi, void *grad_cs);
int lbm_gradient_cs(lbm_ctx *ctx, int T, const int planes[2], void *snapshots, int nsnap, void *lambda,
                    void *grad_phi, void *grad_cs, int mean, double *J, long long *nforward);

/* Number of wall-modeled cells, and their records (host arrays of that
 * length; any pointer may be NULL): cell, reference cell, normal [n][3],
 * and from the last wall prepass u_tau, G, tau_eff.  Synchronises. */
int lbm_wall_count(const lbm_ctx *ctx);

/* Vortex-method inflow perturbation of the velocity inlet (Sec. 2.2.2; needs
 * open_x).  n seed points on the inflow plane: yz host double [n][2], the
 * (y, z) position in cell units (cell j spans [j, j + 1), its centre is
 * j + 1/2; 0 <= y <= ny, 0 <= z <= nz), sign host int [n] (>= 0 for +1, < 0 for -1), turbulence
 * intensity I >= 0, vortex size sigma > 0 (cells).  The library computes
 * k_i = 3/2 (|u_mean(p_i)| I)^2 from the log-law profile at z_i and
 * Gamma_i = 4 s_i sqrt(pi / (6 ln 3 - 9 ln 2) k_i A / n), A = ny nz, and from
 * then on the inlet imposes u_mean(z) x plus
 * u_vortex(x) = 1/(2 pi) sum_i Gamma_i ((p_i - x) x d)(1 - exp(-|x - p_i|^2 /
 * (2 sigma^2))) / |x - p_i|^2 with d = +x (the decaying exponent; the
 * streamwise Langevin term is not applied).  n = 0 restores the mean
 * profile.  0 <= n <= LBM_MAX_VORTICES.  Synchronises the stream (the list
 * is copied into the workspace), then fills the inlet velocity field on it.
 * LBM_EINVAL (nothing changed) for invalid arguments or without open_x. */
enum { LBM_MAX_VORTICES = 4096 };
int lbm_set_inflow_vortices(lbm_ctx *ctx, int n, const double *yz, const int *sign, double intensity,
                            double sigma);
int lbm_wall_records(lbm_ctx *ctx, int *cell, int *ref, double *normal, double *utau, double *G,
                     double *tau);

/* Per-kernel timing of the step kernels with HIP events recorded on the
 * context's stream around each launch: index 0 the separate wall prepass (for
 * wall cells whose reference cell is a wall cell), 1 the bulk
 * collide-and-stream kernel, 2 the wall kernel (records and reconstruction).  lbm_profile(ctx, 1)
 * starts recording (creates the events once), lbm_profile(ctx, 0) stops it;
 * lbm_profile_read waits for the recorded launches and returns, then
 * resets, the accumulated milliseconds and launch counts. */
int lbm_profile(lbm_ctx *ctx, int enable);
int lbm_profile_read(lbm_ctx *ctx, double ms[3], long long count[3]);

/* Memory-system ceiling of the bulk kernel's accesses: n >= 2 launches, at
 * alternating step parity, of a kernel with the bulk kernel's tiles, block
 * order, cell selection and slot map that loads every slot an updated cell
 * reads and stores the value back unchanged (no collision; the state is not
 * modified).  *ms_per_launch receives the mean launch time from HIP events on
 * the context's stream.  The bytes moved per launch are those of the bulk
 * kernel.  Synchronises. */
int lbm_stream_probe(lbm_ctx *ctx, int n, double *ms_per_launch);

/* Host-only inspection of the in-place AA streaming map (Sec. 2.3 stores the
 * populations as structure of arrays; this library updates them in one
 * buffer): builds the cell flags from p and mask (as lbm_init does) and, for
 * every fluid cell c and direction i, gives the slot s = dir * N + cell from
 * which the kernels read f_i(c) (read[i * N + c]) and to which they write
 * f*_i(c) (write[i * N + c]) at step parity `parity` (0 even, 1 odd), using
 * the kernels' own slot functions; -1 at solid cells.  read, write: host
 * int64 [q][N].  No device work; LBM_EINVAL for invalid parameters. */
int lbm_slot_map(const lbm_params *p, const uint8_t *mask, int parity, long long *read, long long *write);

const char *lbm_last_error(const lbm_ctx *ctx);

/* Buffers whose streamed arrays lie far apart in physical memory (for
 * callers that can allocate; any buffer of the right size also works).  The
 * step streams q direction arrays at once; on MI355X that pattern runs at
 * about 65 % of the HBM peak when the arrays are physically adjacent, as one
 * plain allocation places them, and at 75-80 % once they are 3-4 GiB or more
 * apart physically.  These calls cut the buffer into pieces about one array
 * long (whole 2 MiB pages), create each piece as its own physical allocation
 * (virtual memory API) with a temporary spacer allocation after it so that
 * the next lands about 4 GiB further on, release the spacers, and map the
 * pieces back to back into one virtual range: the buffer has the ordinary
 * layout and holds its own size rounded up to whole pieces, but needs up to
 * (q - 1) x 4 GiB of free device memory while it is made.  Arrays of 4 GiB
 * or more are left in one allocation.  Spacers that cannot be made are
 * skipped (the buffer is as correct, possibly slower).
 *  lbm_workspace_alloc: a workspace for lbm_init with these arguments
 *    (*bytes = lbm_workspace_bytes(p, mask, porous)), on the current device,
 *    256-byte aligned, its population arrays spread.
 *  lbm_adjoint_alloc: an adjoint buffer of lbm_adjoint_bytes(ctx) with its
 *    common-mode and deviation arrays spread, zero-filled (synchronous).
 *  lbm_spread_free: releases a buffer of either call (LBM_EINVAL for any
 *    other pointer) after synchronising the device.  A workspace is freed
 *    only after lbm_free of its context.
 * Errors: LBM_EINVAL (invalid parameters, no virtual memory management on
 * the device), LBM_ESIZE (out of device memory), LBM_EHIP. */
int lbm_workspace_alloc(const lbm_params *p, const uint8_t *mask, int porous, void **workspace, size_t *bytes);
int lbm_adjoint_alloc(const lbm_ctx *ctx, void **lambda, size_t *bytes);
int lbm_spread_free(void *ptr);
/* Releases the context (host memory only; the workspace stays the caller's). */
void lbm_free(lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBM_MI355X_H */
