// Internal declarations shared by the host side (abi.cpp, geometry.cpp,
// revolve.cpp) and the device side (kernels.hip, adjoint.hip) of the
// MI355X LBM-LES library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbm.h"

namespace lbmk {

// Per-cell flag byte.  0 = solid (no state).
enum : uint8_t {
  FL_FLUID = 1,  // carries populations
  FL_NEAR = 2,   // at least one link to a solid cell or outside a non-periodic axis
  FL_WALL = 4,   // wall-modeled cell (reconstruction collision, wall kernel)
  FL_LID = 8,    // top-lid cell (inflow equilibrium)
  FL_INLET = 16, // velocity inlet cell (plane x = 0, open x faces)
  FL_OUTLET = 32 // pressure outlet cell (plane x = nx - 1, open x faces)
};

// Number of doubles per wall record (structure of arrays, nwall entries each).
enum {
  WR_NX = 0, WR_NY, WR_NZ,  // unit normal (static)
  WR_YB, WR_YR,             // wall distance of the wall cell and of its reference cell (static)
  WR_TX, WR_TY, WR_TZ,      // unit tangent of the reference velocity (per step)
  WR_UTAN,                  // modeled tangential speed u_tau * u+ at the wall cell (per step)
  WR_G,                     // modeled strain magnitude |S| (per step)
  WR_TAU,                   // effective relaxation time of the wall cell (per step)
  WR_UTAU,                  // friction velocity (per step)
  WR_COUNT
};

// Constants every kernel needs, passed by value.
struct KArgs {
  int nx, ny, nz, N;
  int per[3];
  double tau0;
  double smag;  // 18 sqrt(2) C_S^2: coefficient of |Pi|/rho under the root of tau_eff
  double cs;    // C_S (scalar; the per-cell field csf replaces it when set)
  double cs2;   // C_S^2
  double nu;    // (tau0 - 1/2)/3
  double F[3];
  double kappa, E;
  int fringe_start;  // first fringe plane in x (nx when there is no fringe)
  double u_lid;      // lid velocity (x component)
  int rr;            // 1: recursive regularized collision (third order), 0: BGK
  double fdw;        // weight of the finite-difference strain (1 - sigma), 0 = local only
  int slip;          // full-slip box faces (lbm_params.slip bits)
  int open_x;        // 1: inlet / outlet on the x faces
  double rho_out;    // outlet density
  const void *vel;   // [N] (u_x, u_y, u_z, rho) of the current step at fluid cells, 0 elsewhere, compute type (fdw > 0)
  const void *uin;   // [nz] fringe inflow profile, compute type
  const void *lam;   // [nx] fringe blend weight, compute type (0 before the fringe)
  const void *inflow;  // [3][ny nz] inlet velocity, compute type (open_x)
  const void *csf;     // [N] per-cell Smagorinsky constant C_S, compute type; NULL: C_S^2 = cs2 everywhere
};

// Adjoint field in caller memory (lbm_adjoint_bytes).  The value of a slot is
// M[w] + d[slot]: w is the cell that wrote the slot, M[w] its common mode
// (FP64, one array per layout parity) and d the deviation in the compute type
// (FP64 for FP64 storage, FP32 otherwise).  Two arrays of N doubles, then q
// arrays of N deviations from a 256-byte boundary, then (wall model) four
// doubles per wall record from a 256-byte boundary: the reverse step's
// adjoint of each record's reference-cell density and momentum; then (hybrid
// collision) six arrays of N values in the compute type from a 256-byte
// boundary: the adjoint of each cell's finite-difference strain.
struct AdjLayout {
  size_t d_off, wadj_off, sbar_off, bytes;
};
inline AdjLayout adj_layout(long long N, int q, size_t dev_bytes, long long nwall, bool fd) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  AdjLayout L;
  L.d_off = up((size_t)2 * (size_t)N * sizeof(double));
  L.wadj_off = up(L.d_off + (size_t)q * (size_t)N * dev_bytes);
  size_t end = nwall > 0 ? L.wadj_off + (size_t)4 * (size_t)nwall * sizeof(double) : L.d_off + (size_t)q * (size_t)N * dev_bytes;
  L.sbar_off = up(end);
  if (fd) end = L.sbar_off + (size_t)6 * (size_t)N * dev_bytes;
  L.bytes = end;
  return L;
}

}  // namespace lbmk

namespace lbmk {
// Per-kernel event timing of the step kernels (K1 wall prepass, K2 bulk,
// K3 wall collide), enabled by lbm_profile.  A ring of event pairs per
// kernel; a slot is read back before it is reused.
constexpr int PROF_RING = 256;
struct KernelTimer {
  hipEvent_t start[PROF_RING]{}, stop[PROF_RING]{};
  bool pending[PROF_RING]{};
  int head = 0;
  bool started = false;  // the start event of slot head was recorded
  double ms = 0.0;
  long long count = 0;
};
}  // namespace lbmk

struct lbm_ctx {
  lbm_params p{};
  int q = 0;
  long long N = 0;
  size_t elem = 0;  // bytes per stored population value
  hipStream_t stream = nullptr;
  lbmk::KArgs ka{};
  bool porous = false;
  bool has_solid = false;  // some cell has a solid link (bounce-back needed)
  bool has_slip = false;   // full-slip faces (specular reflection needed)
  bool has_lid = false;
  bool has_open = false;   // some cell is an inlet or outlet cell
  // device regions carved from the caller's workspace
  void *pop = nullptr;        // [q][N] stored deviations
  uint8_t *flags = nullptr;   // [N]
  void *phi = nullptr;        // [N] compute type, porous only
  void *csf = nullptr;        // [N] per-cell C_S, compute type (cs_field only; in force when ka.csf is set)
  void *tables = nullptr;     // [nz] inflow + [nx] fringe weights, compute type
  void *vel = nullptr;        // [N] (u, fluid) vectors, compute type (hybrid collision only)
  void *inflow = nullptr;     // [3][ny nz] inlet velocity, compute type (open_x only)
  double *vort = nullptr;     // [LBM_MAX_VORTICES][3] vortex y, z, circulation (open_x only)
  int nwall = 0;
  int *wcell = nullptr;       // [nwall]
  uint64_t *wmask = nullptr;  // [2][nwall] link masks of the wall cells and of their reference cells
  int *wref = nullptr;        // [nwall]
  uint8_t *wrefwall = nullptr;   // [nwall] 1 when the reference cell is itself a wall cell
  int *wlist_refwall = nullptr;  // [nwall_refwall] indices of those records
  int nwall_refwall = 0;
  // the records grouped by reference cell (for the reverse step): nref
  // distinct reference cells, their records wref_rec[wref_off[u] ..
  // wref_off[u + 1]) in increasing order
  int nref = 0;
  int *wref_cell = nullptr;   // [nref]
  int *wref_off = nullptr;    // [nref + 1]
  int *wref_rec = nullptr;    // [nwall]
  double *wrec = nullptr;     // [WR_COUNT][nwall]
  double *partial = nullptr;  // reduction partials
  int npartial = 0;           // number of partial slots (blocks) available
  double *result = nullptr;   // [8] finalised reductions
  int *errflag = nullptr;     // [1] bit 0 non-finite, bit 1 Newton
  double *scratch = nullptr;  // device address of the static scratch on this context's device
  long long steps = 0;
  std::string err;
  bool profiling = false;
  lbmk::KernelTimer *timers = nullptr;  // [3] when profiling was ever enabled
};

namespace lbmk {

// ---- host geometry (geometry.cpp) ------------------------------------------
struct Geometry {
  std::vector<uint8_t> flags;  // [N]
  std::vector<int> wcell, wref;
  std::vector<double> wnorm;   // [3 * nwall]
  bool has_solid = false;
  bool has_lid = false;
  bool has_open = false;
};
// Builds flags and the wall list; returns LBM_OK or an error code with msg.
int build_geometry(const lbm_params &p, const uint8_t *mask, Geometry &g, std::string &msg);
// Counts wall-modeled cells only (for the workspace size).
long long count_wall_cells(const lbm_params &p, const uint8_t *mask);
// Voxel wall distance of cell c: nearest solid unit cube within two cells.
double voxel_distance(const lbm_params &p, const uint8_t *mask, long long c);

// ---- binomial checkpointing (revolve.cpp) ----------------------------------
enum ActionKind { ACT_ADVANCE, ACT_STORE, ACT_RESTORE, ACT_REVERSE };
struct Action {
  ActionKind kind;
  int arg;   // ADVANCE: number of steps; STORE/RESTORE: slot; REVERSE: step index
  int step;  // step index of the state before the action
};
long long revolve_cost(int T, int nsnap);
std::vector<Action> revolve_schedule(int T, int nsnap);

// ---- device launchers (kernels.hip, adjoint.hip) ---------------------------
// Each returns LBM_OK or LBM_EHIP (with ctx->err set).
int dev_init_equilibrium(lbm_ctx *ctx, const double *rho0, const double *u0);
int dev_inflow(lbm_ctx *ctx, int nvort, double sigma);  // inlet velocity field from ctx->vort
int dev_step(lbm_ctx *ctx);  // one time step at parity ctx->steps & 1
// n launches (alternating parity) of the bulk kernel's access pattern without
// the collision; mean time per launch from events.  Synchronises.
int dev_stream_probe(lbm_ctx *ctx, int n, double *ms_per_launch);
int dev_moments(lbm_ctx *ctx, void *rho, void *u);
// the hybrid's velocity field (ctx->vel) of the current state (fdw > 0)
int dev_velocity4(lbm_ctx *ctx);
int dev_reduce_diag(lbm_ctx *ctx);  // writes result[0..3]
// Looks up (once per device) the address of the static scratch array and
// stores it in ctx->scratch; the current device must be the context's.
int dev_scratch_setup(lbm_ctx *ctx);
// dev_reduce_diag with its partials and sums in the static scratch; *result
// receives the device address of the sums.
int dev_reduce_diag_noalloc(lbm_ctx *ctx, const double **result);
int dev_objective(lbm_ctx *ctx, const int planes[2]);  // writes result[4]
int dev_export(lbm_ctx *ctx, void *f);
int dev_import(lbm_ctx *ctx, const void *f);
int dev_layout_to_natural(lbm_ctx *ctx, const void *lam, void *nat);
int dev_layout_from_natural(lbm_ctx *ctx, const void *nat, void *lam);
// seed of the terminal objective, times w
int dev_adjoint_seed(lbm_ctx *ctx, const int planes[2], void *lam, double w = 1.0);
// one reverse step; seed_w != 0 also adds seed_w dJ/df of the state held
// (planes and the fluid-cell counts of the last objective evaluation);
// gcs != NULL also accumulates dJ/dC_S per cell
int dev_adjoint_step(lbm_ctx *ctx, void *lam, void *grad, void *gcs = nullptr, double seed_w = 0.0,
                     const int *planes = nullptr);
// device buffer of `bytes` whose count arrays [offset + k stride, + stride)
// lie far apart in physical memory, mapped back to back (spread.cpp)
int spread_alloc(size_t bytes, size_t offset, size_t stride, int count, void **out, std::string &msg);
int spread_free(void *ptr);
// copies a device double [N] C_S field into ctx->csf in the compute type;
// *bad != 0 when an entry is negative or not finite (synchronises)
int dev_set_cs(lbm_ctx *ctx, const double *cs, int *bad);
int dev_fill(lbm_ctx *ctx, void *ptr, size_t bytes);  // zero fill with a kernel
int dev_write_header(lbm_ctx *ctx, void *dst);

int hip_fail(lbm_ctx *ctx, hipError_t e, const char *what);
// Event brackets around step kernel k (0: wall prepass, 1: bulk, 2: wall
// step); no-ops unless profiling.
void prof_begin(lbm_ctx *ctx, int k);
void prof_end(lbm_ctx *ctx, int k);

}  // namespace lbmk
