// C ABI of the MI355X LBM-LES library: argument checks, workspace layout,
// geometry upload, the step loop and the checkpointed reverse sweep.  All
// arithmetic of the method runs in the kernels of kernels.hip / adjoint.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "lattice.h"

using namespace lbmk;

namespace {

constexpr size_t ALIGN = 256;
constexpr int PARTIAL_SLOTS = 1024;
constexpr size_t HEADER_BYTES = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

std::string g_static_error;

int set_err(lbm_ctx *ctx, int code, const std::string &msg) {
  if (ctx) ctx->err = msg;
  else g_static_error = msg;
  return code;
}

size_t storage_bytes(int storage) { return storage == LBM_F64 ? 8 : storage == LBM_F32DEV ? 4 : 2; }
size_t compute_bytes(int storage) { return storage == LBM_F64 ? 8 : 4; }

// Parameter validation shared by lbm_workspace_bytes and lbm_init.
bool params_ok(const lbm_params *p, std::string &msg) {
  if (!p) {
    msg = "null parameters";
    return false;
  }
  if (p->lattice != 19 && p->lattice != 27) {
    msg = "lattice must be 19 or 27";
    return false;
  }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) {
    msg = "domain sizes must be positive";
    return false;
  }
  const long long N = (long long)p->nx * p->ny * p->nz;
  if (N >= (1LL << 31)) {
    msg = "domain has 2^31 cells or more";
    return false;
  }
  if (p->storage != LBM_F64 && p->storage != LBM_F32DEV && p->storage != LBM_F16DEV) {
    msg = "storage must be LBM_F64, LBM_F32DEV or LBM_F16DEV";
    return false;
  }
  if ((unsigned long long)N * storage_bytes(p->storage) > (1ULL << 32)) {
    msg = "one population array would exceed 4 GiB (N * bytes per value > 2^32)";
    return false;
  }
  if (!(p->tau0 > 0.5) || !std::isfinite(p->tau0)) {
    msg = "tau0 must be finite and exceed 1/2";
    return false;
  }
  if (!(p->cs_smag >= 0.0) || !std::isfinite(p->cs_smag)) {
    msg = "cs_smag must be finite and >= 0";
    return false;
  }
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->force[a])) {
      msg = "force must be finite";
      return false;
    }
  if (p->wall_model && (!(p->kappa > 0.0) || !(p->E > 0.0))) {
    msg = "wall model needs kappa > 0 and E > 0";
    return false;
  }
  if (p->fringe_len < 0 || p->fringe_len > p->nx) {
    msg = "fringe_len must be in [0, nx]";
    return false;
  }
  if ((p->fringe_len > 0 || p->lid) && (!(p->z0 > 0.0) || !std::isfinite(p->u_ref))) {
    msg = "fringe / lid need z0 > 0 and a finite u_ref";
    return false;
  }
  if (p->collision != LBM_BGK && p->collision != LBM_RR3) {
    msg = "collision must be LBM_BGK or LBM_RR3";
    return false;
  }
  if (!(p->fd_weight >= 0.0 && p->fd_weight <= 1.0) || (p->fd_weight > 0.0 && p->collision != LBM_RR3)) {
    msg = "fd_weight must be in [0, 1], and above 0 only with LBM_RR3";
    return false;
  }
  if (p->open_x != 0 && p->open_x != 1) {
    msg = "open_x must be 0 or 1";
    return false;
  }
  for (int a = 0; a < 3; ++a)
    if (p->periodic[a] && ((p->slip >> (2 * a)) & 3)) {
      msg = "full-slip faces need a non-periodic axis";
      return false;
    }
  if ((p->slip & ~63) || (p->open_x && (p->slip & 3)) || (p->lid && (p->slip & 32))) {
    msg = "slip: six face bits, not on open x faces, not on the top face with a lid";
    return false;
  }
  if (p->open_x && (p->periodic[0] || p->nx < 3 || p->fringe_len > p->nx - 2 || p->fd_weight > 0.0 ||
                    p->force[0] != 0.0 || p->force[1] != 0.0 || p->force[2] != 0.0 || !(p->rho_out > 0.0) ||
                    !std::isfinite(p->rho_out) || !(p->z0 > 0.0) || !std::isfinite(p->u_ref))) {
    msg = "open x faces need a non-periodic x axis, nx >= 3, fringe_len <= nx - 2, no hybrid, no force, "
          "rho_out > 0 and the inflow profile (z0 > 0, finite u_ref)";
    return false;
  }
  return true;
}

struct Layout {
  size_t pop, flags, phi, csf, tables, vel, inflow, vort, wcell, wref, wrefwall, wlist, wrec, wmask, rcell, roff, rrec, partial,
      result, errflag,
      total;
};

Layout layout_of(const lbm_params &p, long long nwall, bool porous) {
  const size_t N = (size_t)p.nx * p.ny * p.nz;
  const size_t rb = compute_bytes(p.storage);
  Layout L{};
  size_t off = 0;
  L.pop = off;
  off += align_up((size_t)p.lattice * N * storage_bytes(p.storage));
  L.flags = off;
  off += align_up(N);
  L.phi = off;
  off += porous ? align_up(N * rb) : 0;
  L.csf = off;
  off += p.cs_field ? align_up(N * rb) : 0;
  L.tables = off;
  off += align_up(((size_t)p.nz + p.nx) * rb);
  L.vel = off;
  off += p.fd_weight > 0.0 ? align_up(4 * N * rb) : 0;
  L.inflow = off;
  off += p.open_x ? align_up(3 * (size_t)p.ny * p.nz * rb) : 0;
  L.vort = off;
  off += p.open_x ? align_up((size_t)LBM_MAX_VORTICES * 3 * sizeof(double)) : 0;
  L.wcell = off;
  off += align_up((size_t)nwall * sizeof(int));
  L.wref = off;
  off += align_up((size_t)nwall * sizeof(int));
  L.wrefwall = off;
  off += align_up((size_t)nwall);
  L.wlist = off;
  off += align_up((size_t)nwall * sizeof(int));
  L.wrec = off;
  off += align_up((size_t)nwall * WR_COUNT * sizeof(double));
  L.wmask = off;
  off += align_up((size_t)nwall * 2 * sizeof(uint64_t));
  // the records grouped by reference cell (reverse step)
  L.rcell = off;
  off += align_up((size_t)nwall * sizeof(int));
  L.roff = off;
  off += align_up(((size_t)nwall + 1) * sizeof(int));
  L.rrec = off;
  off += align_up((size_t)nwall * sizeof(int));
  L.partial = off;
  off += align_up((size_t)PARTIAL_SLOTS * 8 * sizeof(double));
  L.result = off;
  off += align_up(32 * sizeof(double));
  L.errflag = off;
  off += align_up(sizeof(int));
  L.total = off;
  return L;
}

int sync_and_check(lbm_ctx *ctx) {
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  int flag = 0;
  e = hipMemcpy(&flag, ctx->errflag, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "reading the fault flag");
  if (flag & 1) return set_err(ctx, LBM_ENONFINITE, "a cell density became non-finite or non-positive");
  if (flag & 2) return set_err(ctx, LBM_ENEWTON, "wall-function Newton solve failed (no convergence or exp range)");
  return LBM_OK;
}

std::vector<unsigned char> to_compute(const std::vector<double> &v, int storage) {
  std::vector<unsigned char> out(v.size() * compute_bytes(storage));
  if (storage == LBM_F64) std::memcpy(out.data(), v.data(), v.size() * sizeof(double));
  else
    for (size_t i = 0; i < v.size(); ++i) {
      const float f = (float)v[i];
      std::memcpy(out.data() + 4 * i, &f, 4);
    }
  return out;
}

}  // namespace

namespace lbmk {

static void drain_slot(KernelTimer &t, int s) {
  if (!t.pending[s]) return;
  float ms = 0.f;
  if (hipEventSynchronize(t.stop[s]) == hipSuccess && hipEventElapsedTime(&ms, t.start[s], t.stop[s]) == hipSuccess) {
    t.ms += ms;
    t.count += 1;
  }
  t.pending[s] = false;
}

void prof_begin(lbm_ctx *ctx, int k) {
  if (!ctx->profiling) return;
  KernelTimer &t = ctx->timers[k];
  drain_slot(t, t.head);
  t.started = hipEventRecord(t.start[t.head], ctx->stream) == hipSuccess;
}

void prof_end(lbm_ctx *ctx, int k) {
  if (!ctx->profiling) return;
  KernelTimer &t = ctx->timers[k];
  // A launch whose events could not both be recorded is left out of the sums.
  if (!t.started || hipEventRecord(t.stop[t.head], ctx->stream) != hipSuccess) return;
  t.started = false;
  t.pending[t.head] = true;
  t.head = (t.head + 1) % PROF_RING;
}

}  // namespace lbmk

namespace {
// Link masks of the wall cells (wm[w]) and of their reference cells
// (wm[nwall + w], 0 unless the reference cell has a solid link), as the
// kernels' solid_mask gives them; the geometry is static, so the wall kernels
// read them instead of gathering the neighbours' flags every odd step.
template <int Q, bool SLIP>
void wall_masks(const KArgs &k, const uint8_t *flags, const std::vector<int> &wcell, const std::vector<int> &wref,
                std::vector<uint64_t> &wm) {
  const size_t M = wcell.size();
  auto mask_of = [&](int c) {
    int x, y, z;
    cell_xyz(c, k, x, y, z);
    return (uint64_t)solid_mask<Q, SLIP>(make_nb(x, y, z, k), flags);
  };
  for (size_t w = 0; w < M; ++w) {
    wm[w] = mask_of(wcell[w]);
    wm[M + w] = (flags[wref[w]] & FL_NEAR) ? mask_of(wref[w]) : 0u;
  }
}

// Slots of every fluid cell at one parity, by the kernels' own slot
// functions: the plain path for cells without solid links (every cell at
// even parity), the bounce-back map for the others.
template <int Q, bool ODD, bool SLIP>
void slot_map_q(const KArgs &k, const uint8_t *flags, long long *rd, long long *wr) {
  const long long N = k.N;
  for (long long c = 0; c < N; ++c) {
    if (!(flags[c] & FL_FLUID)) {
      for (int i = 0; i < Q; ++i) rd[i * N + c] = wr[i * N + c] = -1;
      continue;
    }
    int x, y, z;
    cell_xyz((int)c, k, x, y, z);
    const Nb n = make_nb(x, y, z, k);
    const LinkMask sm = (ODD && (flags[c] & FL_NEAR)) ? solid_mask<Q, SLIP>(n, flags) : 0u;
    for (int i = 0; i < Q; ++i) {
      if (sm != 0u) {
        rd[i * N + c] = (long long)read_slot<Q, ODD, SLIP>(n, sm, i, (size_t)N);
        wr[i * N + c] = (long long)write_slot<Q, ODD, SLIP>(n, sm, i, (size_t)N);
      } else {
        int dr, dw;
        const int ir = plain_read<Q, ODD>(n, i, dr), iw = plain_write<Q, ODD>(n, i, dw);
        rd[i * N + c] = (long long)dr * N + ir;
        wr[i * N + c] = (long long)dw * N + iw;
      }
    }
  }
}
}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_params *p, const uint8_t *mask, int porous) {
  std::string msg;
  if (!params_ok(p, msg)) {
    g_static_error = msg;
    return 0;
  }
  return layout_of(*p, count_wall_cells(*p, mask), porous != 0).total;
}

int lbm_init(lbm_ctx **out, const lbm_params *p, const uint8_t *mask, const double *wall_dist,
             const double *porosity, const double *rho0, const double *u0, void *workspace,
             size_t workspace_bytes) {
  std::string msg;
  if (!out) return set_err(nullptr, LBM_EINVAL, "null output pointer");
  *out = nullptr;
  if (!params_ok(p, msg)) return set_err(nullptr, LBM_EINVAL, msg);
  if (!workspace || ((uintptr_t)workspace % ALIGN) != 0)
    return set_err(nullptr, LBM_EINVAL, "workspace must be non-null and 256-byte aligned");
  const long long N = (long long)p->nx * p->ny * p->nz;
  if (porosity)
    for (long long c = 0; c < N; ++c)
      if (!(porosity[c] >= 0.0 && porosity[c] <= 1.0))
        return set_err(nullptr, LBM_EINVAL, "porosity must lie in [0, 1]");

  Geometry g;
  int rc = build_geometry(*p, mask, g, msg);
  if (rc != LBM_OK) return set_err(nullptr, rc, msg);
  const long long nwall = (long long)g.wcell.size();
  const Layout L = layout_of(*p, nwall, porosity != nullptr);
  if (workspace_bytes < L.total)
    return set_err(nullptr, LBM_ESIZE, "workspace smaller than lbm_workspace_bytes()");

  // wall records: normals and wall distances (static part)
  std::vector<double> rec((size_t)nwall * WR_COUNT, 0.0);
  for (long long k = 0; k < nwall; ++k) {
    const long long b = g.wcell[k], r = g.wref[k];
    const double yb = wall_dist ? wall_dist[b] : voxel_distance(*p, mask, b);
    const double yr = wall_dist ? wall_dist[r] : voxel_distance(*p, mask, r);
    if (!(yb > 0.0 && std::isfinite(yb) && yr > 0.0 && std::isfinite(yr)))
      return set_err(nullptr, LBM_EINVAL,
                     "wall distance must be positive and finite at wall cells and their references");
    for (int a = 0; a < 3; ++a) rec[(size_t)(WR_NX + a) * nwall + k] = g.wnorm[3 * k + a];
    rec[(size_t)WR_YB * nwall + k] = yb;
    rec[(size_t)WR_YR * nwall + k] = yr;
    rec[(size_t)WR_TAU * nwall + k] = p->tau0;
  }

  lbm_ctx *ctx = new (std::nothrow) lbm_ctx();
  if (!ctx) return set_err(nullptr, LBM_EINVAL, "out of host memory");
  ctx->p = *p;
  ctx->q = p->lattice;
  ctx->N = N;
  ctx->elem = storage_bytes(p->storage);
  ctx->stream = (hipStream_t)p->stream;
  ctx->porous = porosity != nullptr;
  ctx->has_solid = g.has_solid;
  ctx->has_slip = p->slip != 0 && g.has_solid;
  ctx->has_lid = g.has_lid;
  ctx->has_open = g.has_open;
  char *base = (char *)workspace;
  ctx->pop = base + L.pop;
  ctx->flags = (uint8_t *)(base + L.flags);
  ctx->phi = ctx->porous ? base + L.phi : nullptr;
  ctx->csf = p->cs_field ? base + L.csf : nullptr;
  ctx->tables = base + L.tables;
  ctx->vel = p->fd_weight > 0.0 ? base + L.vel : nullptr;
  ctx->inflow = p->open_x ? base + L.inflow : nullptr;
  ctx->vort = p->open_x ? (double *)(base + L.vort) : nullptr;
  ctx->nwall = (int)nwall;
  ctx->wcell = (int *)(base + L.wcell);
  ctx->wref = (int *)(base + L.wref);
  ctx->wrefwall = (uint8_t *)(base + L.wrefwall);
  ctx->wlist_refwall = (int *)(base + L.wlist);
  ctx->wref_cell = (int *)(base + L.rcell);
  ctx->wref_off = (int *)(base + L.roff);
  ctx->wref_rec = (int *)(base + L.rrec);
  ctx->wrec = (double *)(base + L.wrec);
  ctx->wmask = (uint64_t *)(base + L.wmask);
  ctx->partial = (double *)(base + L.partial);
  ctx->npartial = PARTIAL_SLOTS;
  ctx->result = (double *)(base + L.result);
  ctx->errflag = (int *)(base + L.errflag);

  // kernel constants
  KArgs &k = ctx->ka;
  k.nx = p->nx;
  k.ny = p->ny;
  k.nz = p->nz;
  k.N = (int)N;
  for (int a = 0; a < 3; ++a) k.per[a] = p->periodic[a] ? 1 : 0;
  k.tau0 = p->tau0;
  k.cs = p->cs_smag;
  k.cs2 = p->cs_smag * p->cs_smag;
  k.csf = nullptr;
  k.smag = 18.0 * std::sqrt(2.0) * k.cs2;
  k.nu = (p->tau0 - 0.5) / 3.0;
  for (int a = 0; a < 3; ++a) k.F[a] = p->force[a];
  k.kappa = p->kappa;
  k.E = p->E;
  k.fringe_start = p->fringe_len > 0 ? p->nx - p->fringe_len : p->nx;
  k.u_lid = p->u_ref;  // ln(1 + z_top/z0) / ln(1 + z_top/z0) = 1 at the lid plane
  k.rr = p->collision == LBM_RR3 ? 1 : 0;
  k.fdw = p->fd_weight;
  k.vel = p->fd_weight > 0.0 ? ctx->vel : nullptr;
  k.open_x = p->open_x;
  k.slip = p->slip;
  k.inflow = ctx->inflow;
  k.rho_out = p->open_x ? p->rho_out : 1.0;
  // inflow profile u_in(z) and fringe weights lambda(x)
  std::vector<double> tab((size_t)p->nz + p->nx, 0.0);
  if (p->fringe_len > 0 || p->lid || p->open_x) {
    const double ztop = p->nz - 0.5;
    for (int z = 0; z < p->nz; ++z)
      tab[z] = p->u_ref * std::log(1.0 + (z + 0.5) / p->z0) / std::log(1.0 + ztop / p->z0);
  }
  for (int x = k.fringe_start; x < p->nx; ++x) {
    const double s = double(x - k.fringe_start + 1) / p->fringe_len;
    tab[(size_t)p->nz + x] = s * s * (3.0 - 2.0 * s);
  }
  std::vector<unsigned char> tabc = to_compute(tab, p->storage);
  k.uin = ctx->tables;
  k.lam = (char *)ctx->tables + (size_t)p->nz * compute_bytes(p->storage);

  hipError_t e;
  auto fail = [&](hipError_t err, const char *what) {
    int code = hip_fail(ctx, err, what);
    g_static_error = ctx->err;
    delete ctx;
    return code;
  };
  std::vector<unsigned char> phic;
  if (porosity) {
    std::vector<double> ph(porosity, porosity + N);
    phic = to_compute(ph, p->storage);
  }
  // uploads (synchronous copies from pageable host memory; the stream is
  // synchronised below before any kernel reads them)
  if ((e = hipMemcpy(ctx->flags, g.flags.data(), (size_t)N, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e, "upload flags");
  if ((e = hipMemcpy(ctx->tables, tabc.data(), tabc.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e, "upload tables");
  if (porosity && (e = hipMemcpy(ctx->phi, phic.data(), phic.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e, "upload porosity");
  if (nwall > 0) {
    // records whose reference cell is a wall cell get their own prepass launch
    std::vector<uint8_t> refwall((size_t)nwall, 0);
    std::vector<int> list;
    for (long long k = 0; k < nwall; ++k)
      if (g.flags[(size_t)g.wref[k]] & FL_WALL) {
        refwall[k] = 1;
        list.push_back((int)k);
      }
    ctx->nwall_refwall = (int)list.size();
    if ((e = hipMemcpy(ctx->wrefwall, refwall.data(), (size_t)nwall, hipMemcpyHostToDevice)) != hipSuccess)
      return fail(e, "upload wall reference classes");
    if (!list.empty() &&
        (e = hipMemcpy(ctx->wlist_refwall, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice)) !=
            hipSuccess)
      return fail(e, "upload wall reference list");
    if ((e = hipMemcpy(ctx->wcell, g.wcell.data(), nwall * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
      return fail(e, "upload wall cells");
    if ((e = hipMemcpy(ctx->wref, g.wref.data(), nwall * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
      return fail(e, "upload wall references");
    if ((e = hipMemcpy(ctx->wrec, rec.data(), rec.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
      return fail(e, "upload wall records");
    // link masks of each wall cell and of its reference cell (static geometry)
    std::vector<uint64_t> wm((size_t)2 * nwall);
    if (ctx->q == 19) {
      if (ctx->has_slip) wall_masks<19, true>(k, g.flags.data(), g.wcell, g.wref, wm);
      else wall_masks<19, false>(k, g.flags.data(), g.wcell, g.wref, wm);
    } else {
      if (ctx->has_slip) wall_masks<27, true>(k, g.flags.data(), g.wcell, g.wref, wm);
      else wall_masks<27, false>(k, g.flags.data(), g.wcell, g.wref, wm);
    }
    if ((e = hipMemcpy(ctx->wmask, wm.data(), wm.size() * sizeof(uint64_t), hipMemcpyHostToDevice)) != hipSuccess)
      return fail(e, "upload wall link masks");
    // records grouped by reference cell, in increasing cell and record order
    std::vector<int> order((size_t)nwall);
    for (long long k = 0; k < nwall; ++k) order[(size_t)k] = (int)k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return g.wref[a] < g.wref[b]; });
    std::vector<int> rcell, roff;
    for (size_t j = 0; j < order.size(); ++j)
      if (j == 0 || g.wref[order[j]] != g.wref[order[j - 1]]) {
        rcell.push_back(g.wref[order[j]]);
        roff.push_back((int)j);
      }
    roff.push_back((int)nwall);
    ctx->nref = (int)rcell.size();
    if ((e = hipMemcpy(ctx->wref_cell, rcell.data(), rcell.size() * sizeof(int), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(ctx->wref_off, roff.data(), roff.size() * sizeof(int), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(ctx->wref_rec, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice)) !=
            hipSuccess)
      return fail(e, "upload wall reference groups");
  }
  if (dev_scratch_setup(ctx) != LBM_OK || dev_fill(ctx, ctx->errflag, ALIGN) != LBM_OK ||
      (p->open_x && dev_inflow(ctx, 0, 1.0) != LBM_OK) ||
      dev_init_equilibrium(ctx, rho0, u0) != LBM_OK) {
    int code = LBM_EHIP;
    g_static_error = ctx->err;
    delete ctx;
    return code;
  }
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return fail(e, "hipStreamSynchronize");
  ctx->steps = 0;
  *out = ctx;
  return LBM_OK;
}

int lbm_step(lbm_ctx *ctx, int n) {
  if (!ctx) return LBM_EINVAL;
  if (n < 0) return set_err(ctx, LBM_EINVAL, "negative step count");
  for (int s = 0; s < n; ++s) {
    int rc = dev_step(ctx);
    if (rc != LBM_OK) return rc;
    ++ctx->steps;
  }
  return LBM_OK;
}

int lbm_moments(lbm_ctx *ctx, void *rho, void *u) {
  if (!ctx) return LBM_EINVAL;
  if (!rho && !u) return set_err(ctx, LBM_EINVAL, "both outputs are null");
  return dev_moments(ctx, rho, u);
}

int lbm_sync(lbm_ctx *ctx) {
  if (!ctx) return LBM_EINVAL;
  return sync_and_check(ctx);
}

int lbm_diagnostics(lbm_ctx *ctx, double out[4]) {
  if (!ctx || !out) return ctx ? set_err(ctx, LBM_EINVAL, "null output") : LBM_EINVAL;
  int rc = dev_reduce_diag(ctx);
  if (rc != LBM_OK) return rc;
  rc = sync_and_check(ctx);
  if (rc != LBM_OK) return rc;
  double r[8];
  hipError_t e = hipMemcpy(r, ctx->result, sizeof(r), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "read diagnostics");
  // mass = number of fluid cells + sum of density deviations
  out[0] = r[4] + r[0];
  out[1] = r[1];
  out[2] = r[2];
  out[3] = r[3];
  return LBM_OK;
}

int lbm_diagnostics_noalloc(lbm_ctx *ctx, double out[4]) {
  if (!ctx || !out) return ctx ? set_err(ctx, LBM_EINVAL, "null output") : LBM_EINVAL;
  const double *res = nullptr;
  int rc = dev_reduce_diag_noalloc(ctx, &res);
  if (rc != LBM_OK) return rc;
  rc = sync_and_check(ctx);
  if (rc != LBM_OK) return rc;
  double r[8];
  hipError_t e = hipMemcpy(r, res, sizeof(r), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "read diagnostics");
  out[0] = r[4] + r[0];
  out[1] = r[1];
  out[2] = r[2];
  out[3] = r[3];
  return LBM_OK;
}

long long lbm_steps_done(const lbm_ctx *ctx) { return ctx ? ctx->steps : -1; }

int lbm_shape(const lbm_ctx *ctx, int out[5]) {
  if (!ctx || !out) return LBM_EINVAL;
  out[0] = ctx->q;
  out[1] = ctx->p.nx;
  out[2] = ctx->p.ny;
  out[3] = ctx->p.nz;
  out[4] = ctx->p.storage;
  return LBM_OK;
}

int lbm_get_populations(lbm_ctx *ctx, void *f) {
  if (!ctx || !f) return ctx ? set_err(ctx, LBM_EINVAL, "null output") : LBM_EINVAL;
  return dev_export(ctx, f);
}

int lbm_set_populations(lbm_ctx *ctx, const void *f) {
  if (!ctx || !f) return ctx ? set_err(ctx, LBM_EINVAL, "null input") : LBM_EINVAL;
  return dev_import(ctx, f);
}

size_t lbm_state_bytes(const lbm_ctx *ctx) {
  if (!ctx) return 0;
  return HEADER_BYTES + align_up((size_t)ctx->q * ctx->N * ctx->elem);
}

int lbm_save_state(lbm_ctx *ctx, void *dst) {
  if (!ctx || !dst) return ctx ? set_err(ctx, LBM_EINVAL, "null destination") : LBM_EINVAL;
  int rc = dev_write_header(ctx, dst);
  if (rc != LBM_OK) return rc;
  hipError_t e = hipMemcpyAsync((char *)dst + HEADER_BYTES, ctx->pop, (size_t)ctx->q * ctx->N * ctx->elem,
                                hipMemcpyDeviceToDevice, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "save state");
  return LBM_OK;
}

int lbm_load_state(lbm_ctx *ctx, const void *src) {
  if (!ctx || !src) return ctx ? set_err(ctx, LBM_EINVAL, "null source") : LBM_EINVAL;
  long long h[5];
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  e = hipMemcpy(h, src, sizeof(h), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "read state header");
  if (h[0] != 0x4c424d5354415445LL || h[2] != ctx->q || h[3] != ctx->N || h[4] != ctx->p.storage)
    return set_err(ctx, LBM_EINVAL, "state buffer does not match this context");
  e = hipMemcpyAsync(ctx->pop, (const char *)src + HEADER_BYTES, (size_t)ctx->q * ctx->N * ctx->elem,
                     hipMemcpyDeviceToDevice, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "load state");
  ctx->steps = h[1];
  return LBM_OK;
}

int lbm_objective(lbm_ctx *ctx, const int planes[2], double *J) {
  if (!ctx || !planes || !J) return ctx ? set_err(ctx, LBM_EINVAL, "null argument") : LBM_EINVAL;
  if (planes[0] < 0 || planes[0] >= ctx->p.nx || planes[1] < 0 || planes[1] >= ctx->p.nx)
    return set_err(ctx, LBM_EINVAL, "objective planes outside the domain");
  int rc = dev_objective(ctx, planes);
  if (rc != LBM_OK) return rc;
  rc = sync_and_check(ctx);
  if (rc != LBM_OK) return rc;
  double r[8];
  hipError_t e = hipMemcpy(r, ctx->result + 8, sizeof(r), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "read objective");
  const double n0 = r[3], n1 = r[4], nf = r[5];
  if (!(n0 > 0) || !(n1 > 0) || !(nf > 0)) return set_err(ctx, LBM_EINVAL, "objective planes hold no fluid cell");
  *J = (1.0 / 3.0) * (r[0] / n0 - r[1] / n1) + r[2] / nf;
  return LBM_OK;
}

size_t lbm_adjoint_bytes(const lbm_ctx *ctx) {
  if (!ctx) return 0;
  return adj_layout(ctx->N, ctx->q, ctx->p.storage == LBM_F64 ? 8 : 4, ctx->nwall, ctx->ka.fdw > 0.0).bytes;
}

static bool adj_aligned(const void *p) { return ((uintptr_t)p & 7u) == 0; }

int lbm_adjoint_seed(lbm_ctx *ctx, const int planes[2], void *lambda) {
  if (!ctx || !planes || !lambda) return ctx ? set_err(ctx, LBM_EINVAL, "null argument") : LBM_EINVAL;
  if (planes[0] < 0 || planes[0] >= ctx->p.nx || planes[1] < 0 || planes[1] >= ctx->p.nx)
    return set_err(ctx, LBM_EINVAL, "objective planes outside the domain");
  if (!adj_aligned(lambda)) return set_err(ctx, LBM_EINVAL, "adjoint buffer not 8-byte aligned");
  return dev_adjoint_seed(ctx, planes, lambda);
}

int lbm_adjoint_step_cs(lbm_ctx *ctx, void *lambda, void *grad_phi, void *grad_cs) {
  if (!ctx || !lambda || !grad_phi) return ctx ? set_err(ctx, LBM_EINVAL, "null argument") : LBM_EINVAL;
  if (!adj_aligned(lambda) || !adj_aligned(grad_phi) || !adj_aligned(grad_cs))
    return set_err(ctx, LBM_EINVAL, "adjoint or gradient buffer not 8-byte aligned");
  return dev_adjoint_step(ctx, lambda, grad_phi, grad_cs);
}

int lbm_adjoint_step(lbm_ctx *ctx, void *lambda, void *grad_phi) {
  return lbm_adjoint_step_cs(ctx, lambda, grad_phi, nullptr);
}

int lbm_set_smagorinsky(lbm_ctx *ctx, const double *cs) {
  if (!ctx) return LBM_EINVAL;
  if (!ctx->csf) return set_err(ctx, LBM_EINVAL, "no room for a C_S field: create the context with cs_field = 1");
  if (!cs) {
    ctx->ka.csf = nullptr;
    return LBM_OK;
  }
  if (((uintptr_t)cs & 7u) != 0) return set_err(ctx, LBM_EINVAL, "C_S field not 8-byte aligned");
  int bad = 0;
  const int rc = dev_set_cs(ctx, cs, &bad);
  if (rc != LBM_OK) return rc;
  if (bad) return set_err(ctx, LBM_EINVAL, "C_S must be finite and >= 0 at every cell");
  ctx->ka.csf = ctx->csf;
  return LBM_OK;
}

int lbm_adjoint_to_natural(lbm_ctx *ctx, const void *lambda, void *natural) {
  if (!ctx || !lambda || !natural) return ctx ? set_err(ctx, LBM_EINVAL, "null argument") : LBM_EINVAL;
  if (!adj_aligned(lambda) || !adj_aligned(natural)) return set_err(ctx, LBM_EINVAL, "buffer not 8-byte aligned");
  return dev_layout_to_natural(ctx, lambda, natural);
}

int lbm_adjoint_from_natural(lbm_ctx *ctx, const void *natural, void *lambda) {
  if (!ctx || !lambda || !natural) return ctx ? set_err(ctx, LBM_EINVAL, "null argument") : LBM_EINVAL;
  if (!adj_aligned(lambda) || !adj_aligned(natural)) return set_err(ctx, LBM_EINVAL, "buffer not 8-byte aligned");
  return dev_layout_from_natural(ctx, natural, lambda);
}

long long lbm_revolve_cost(int T, int nsnap) { return revolve_cost(T, nsnap); }

// Checkpointed reverse sweep for the terminal objective J = j(f_T) or, with
// mean, the time average J = (1/T) sum_{t=1..T} j(f_t).  The average's
// forward values are summed on the schedule's first descent (the first time
// each step index is reached); its seeds enter the reverse steps t = T-1 .. 1
// fused into the adjoint kernel, and the terminal seed is scaled by 1/T.
static int gradient_sweep(lbm_ctx *ctx, int T, const int planes[2], void *snapshots, int nsnap, void *lambda,
                          void *grad_phi, void *grad_cs, double *J, long long *nforward, bool mean) {
  if (!ctx) return LBM_EINVAL;
  if (T < 1 || nsnap < 1 || !snapshots || !lambda || !grad_phi || !planes)
    return set_err(ctx, LBM_EINVAL, "gradient needs T >= 1, nsnap >= 1 and non-null buffers");
  if (!adj_aligned(lambda) || !adj_aligned(grad_phi) || !adj_aligned(grad_cs))
    return set_err(ctx, LBM_EINVAL, "adjoint or gradient buffer not 8-byte aligned");
  const size_t sb = lbm_state_bytes(ctx);
  auto slot = [&](int k) { return (char *)snapshots + (size_t)k * sb; };
  long long fwd = 0;
  int rc = lbm_save_state(ctx, slot(0));
  if (rc != LBM_OK) return rc;
  const long long step0 = ctx->steps;
  if ((rc = dev_fill(ctx, grad_phi, (size_t)ctx->N * sizeof(double))) != LBM_OK) return rc;
  if (grad_cs && (rc = dev_fill(ctx, grad_cs, (size_t)ctx->N * sizeof(double))) != LBM_OK) return rc;
  // The binomial schedule's first descent is the forward sweep: it stores
  // its checkpoints on the way to step T-1.  There, one more step gives the
  // final state for the objective and the seed; then the last restored
  // checkpoint is advanced back to T-1 and the reverse sweep starts.
  const std::vector<Action> acts = revolve_schedule(T, nsnap);
  long long have = 0;  // step index held by the context, relative to step0
  long long seen = 0;  // largest step index reached so far
  int last_slot = 0;
  long long last_step = 0;
  bool seeded = false;
  double Jv = 0.0, Jsum = 0.0;
  const double w = mean ? 1.0 / T : 1.0;
  for (const Action &a : acts) {
    switch (a.kind) {
      case ACT_RESTORE:
        last_slot = a.arg;
        last_step = a.step;
        if (have != a.step) {
          if ((rc = lbm_load_state(ctx, slot(a.arg))) != LBM_OK) return rc;
          have = a.step;
        }
        break;
      case ACT_ADVANCE:
        if (mean && have + a.arg > seen) {
          // one step at a time through states not seen yet, summing j(f_t)
          for (int s = 0; s < a.arg; ++s) {
            if ((rc = lbm_step(ctx, 1)) != LBM_OK) return rc;
            ++fwd;
            if (++have > seen) {
              double jt;
              if ((rc = lbm_objective(ctx, planes, &jt)) != LBM_OK) return rc;
              Jsum += jt;
              seen = have;
            }
          }
          break;
        }
        if ((rc = lbm_step(ctx, a.arg)) != LBM_OK) return rc;
        fwd += a.arg;
        have += a.arg;
        break;
      case ACT_STORE:
        if ((rc = lbm_save_state(ctx, slot(a.arg))) != LBM_OK) return rc;
        break;
      case ACT_REVERSE:
        if (!seeded) {
          if (a.arg != T - 1 || have != T - 1) return set_err(ctx, LBM_EINVAL, "internal: schedule out of step");
          if ((rc = lbm_step(ctx, 1)) != LBM_OK) return rc;
          fwd += 1;
          if ((rc = lbm_objective(ctx, planes, &Jv)) != LBM_OK) return rc;
          Jsum += Jv;
          if ((rc = dev_adjoint_seed(ctx, planes, lambda, w)) != LBM_OK) return rc;
          if ((rc = lbm_load_state(ctx, slot(last_slot))) != LBM_OK) return rc;
          if (T - 1 > last_step) {
            if ((rc = lbm_step(ctx, (int)(T - 1 - last_step))) != LBM_OK) return rc;
            fwd += T - 1 - last_step;
          }
          have = T - 1;
          seeded = true;
        }
        if (ctx->steps != step0 + a.arg) return set_err(ctx, LBM_EINVAL, "internal: schedule out of step");
        // the seed of step t (t >= 1) joins the reverse step that produces dJ/df_t
        if ((rc = dev_adjoint_step(ctx, lambda, grad_phi, grad_cs, mean && a.arg >= 1 ? w : 0.0, planes)) !=
            LBM_OK)
          return rc;
        break;
    }
  }
  if ((rc = lbm_load_state(ctx, slot(0))) != LBM_OK) return rc;
  if ((rc = sync_and_check(ctx)) != LBM_OK) return rc;
  if (J) *J = mean ? Jsum / T : Jv;
  if (nforward) *nforward = fwd;
  return LBM_OK;
}

int lbm_gradient(lbm_ctx *ctx, int T, const int planes[2], void *snapshots, int nsnap, void *lambda,
                 void *grad_phi, double *J, long long *nforward) {
  return gradient_sweep(ctx, T, planes, snapshots, nsnap, lambda, grad_phi, nullptr, J, nforward, false);
}

int lbm_gradient_mean(lbm_ctx *ctx, int T, const int planes[2], void *snapshots, int nsnap, void *lambda,
                      void *grad_phi, double *J, long long *nforward) {
  return gradient_sweep(ctx, T, planes, snapshots, nsnap, lambda, grad_phi, nullptr, J, nforward, true);
}

int lbm_gradient_cs(lbm_ctx *ctx, int T, const int planes[2], void *snapshots, int nsnap, void *lambda,
                    void *grad_phi, void *grad_cs, int mean, double *J, long long *nforward) {
  if (!ctx) return LBM_EINVAL;
  if (!grad_cs) return set_err(ctx, LBM_EINVAL, "null C_S gradient buffer");
  return gradient_sweep(ctx, T, planes, snapshots, nsnap, lambda, grad_phi, grad_cs, J, nforward, mean != 0);
}

int lbm_wall_count(const lbm_ctx *ctx) { return ctx ? ctx->nwall : -1; }

int lbm_set_inflow_vortices(lbm_ctx *ctx, int n, const double *yz, const int *sign, double intensity,
                            double sigma) {
  if (!ctx) return LBM_EINVAL;
  if (!ctx->p.open_x) return set_err(ctx, LBM_EINVAL, "vortices need open x faces");
  if (n < 0 || n > LBM_MAX_VORTICES || (n > 0 && (!yz || !sign)))
    return set_err(ctx, LBM_EINVAL, "vortex count must be in [0, LBM_MAX_VORTICES] with positions and signs");
  if (!(sigma > 0.0) || !std::isfinite(sigma) || !(intensity >= 0.0) || !std::isfinite(intensity))
    return set_err(ctx, LBM_EINVAL, "vortices need sigma > 0 and intensity >= 0, both finite");
  for (int i = 0; i < n; ++i)
    if (!(yz[2 * i] >= 0.0 && yz[2 * i] <= ctx->p.ny && yz[2 * i + 1] >= 0.0 && yz[2 * i + 1] <= ctx->p.nz))
      return set_err(ctx, LBM_EINVAL, "vortex positions must lie on the inflow plane, 0 <= y <= ny, 0 <= z <= nz");
  // circulations: k_i = 3/2 (|u_mean(z_i)| I)^2, Gamma_i = 4 s_i sqrt(pi / (6 ln 3 - 9 ln 2) k_i A / n)
  const double pi = 3.14159265358979323846;
  const double A = (double)ctx->p.ny * ctx->p.nz;
  const double ztop = ctx->p.nz - 0.5;
  std::vector<double> v((size_t)3 * n);
  for (int i = 0; i < n; ++i) {
    const double z = yz[2 * i + 1];
    const double um = std::fabs(ctx->p.u_ref * std::log(1.0 + z / ctx->p.z0) / std::log(1.0 + ztop / ctx->p.z0));
    const double k = 1.5 * (um * intensity) * (um * intensity);
    v[3 * i] = yz[2 * i];
    v[3 * i + 1] = z;
    const double c = pi / (6.0 * std::log(3.0) - 9.0 * std::log(2.0));
    v[3 * i + 2] = 4.0 * (sign[i] >= 0 ? 1.0 : -1.0) * std::sqrt(c * k * A / n);
  }
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  if (n > 0 && (e = hipMemcpy(ctx->vort, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(ctx, e, "upload vortices");
  return dev_inflow(ctx, n, sigma);
}

int lbm_wall_records(lbm_ctx *ctx, int *cell, int *ref, double *normal, double *utau, double *G, double *tau) {
  if (!ctx) return LBM_EINVAL;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  const size_t nw = (size_t)ctx->nwall;
  if (nw == 0) return LBM_OK;
  std::vector<double> rec(nw * WR_COUNT);
  if ((e = hipMemcpy(rec.data(), ctx->wrec, rec.size() * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(ctx, e, "read wall records");
  if (cell && (e = hipMemcpy(cell, ctx->wcell, nw * sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(ctx, e, "read wall cells");
  if (ref && (e = hipMemcpy(ref, ctx->wref, nw * sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(ctx, e, "read wall references");
  for (size_t k = 0; k < nw; ++k) {
    if (normal)
      for (int a = 0; a < 3; ++a) normal[3 * k + a] = rec[(WR_NX + a) * nw + k];
    if (utau) utau[k] = rec[WR_UTAU * nw + k];
    if (G) G[k] = rec[WR_G * nw + k];
    if (tau) tau[k] = rec[WR_TAU * nw + k];
  }
  return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *ctx) { return ctx ? ctx->err.c_str() : g_static_error.c_str(); }

int lbm_workspace_alloc(const lbm_params *p, const uint8_t *mask, int porous, void **workspace, size_t *bytes) {
  if (!workspace || !bytes) return set_err(nullptr, LBM_EINVAL, "null output pointer");
  *workspace = nullptr;
  *bytes = 0;
  const size_t need = lbm_workspace_bytes(p, mask, porous);
  if (need == 0) return LBM_EINVAL;  // lbm_workspace_bytes left the message
  const size_t N = (size_t)p->nx * p->ny * p->nz;
  std::string msg;
  const int rc = spread_alloc(need, 0, N * storage_bytes(p->storage), p->lattice, workspace, msg);
  if (rc != LBM_OK) return set_err(nullptr, rc, msg);
  *bytes = need;
  return LBM_OK;
}

int lbm_adjoint_alloc(const lbm_ctx *ctx, void **lambda, size_t *bytes) {
  if (!ctx || !lambda || !bytes) return set_err(nullptr, LBM_EINVAL, "null argument");
  *lambda = nullptr;
  *bytes = 0;
  const size_t db = ctx->p.storage == LBM_F64 ? 8 : 4;
  const AdjLayout L = adj_layout(ctx->N, ctx->q, db, ctx->nwall, ctx->ka.fdw > 0.0);
  std::string msg;
  const int rc = spread_alloc(L.bytes, L.d_off, (size_t)ctx->N * db, ctx->q, lambda, msg);
  if (rc != LBM_OK) return set_err(nullptr, rc, msg);
  const hipError_t e = hipMemset(*lambda, 0, L.bytes);
  if (e != hipSuccess) {
    (void)spread_free(*lambda);
    *lambda = nullptr;
    return set_err(nullptr, LBM_EHIP, std::string("hipMemset of the adjoint buffer: ") + hipGetErrorString(e));
  }
  *bytes = L.bytes;
  return LBM_OK;
}

int lbm_spread_free(void *ptr) {
  if (spread_free(ptr) != LBM_OK) return set_err(nullptr, LBM_EINVAL, "not a buffer of lbm_workspace_alloc / lbm_adjoint_alloc");
  return LBM_OK;
}

int lbm_profile(lbm_ctx *ctx, int enable) {
  if (!ctx) return LBM_EINVAL;
  if (enable && !ctx->timers) {
    ctx->timers = new (std::nothrow) KernelTimer[3];
    if (!ctx->timers) return set_err(ctx, LBM_EINVAL, "out of host memory");
    for (int k = 0; k < 3; ++k)
      for (int s = 0; s < PROF_RING; ++s) {
        hipError_t e = hipEventCreate(&ctx->timers[k].start[s]);
        if (e == hipSuccess) e = hipEventCreate(&ctx->timers[k].stop[s]);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventCreate");
      }
  }
  ctx->profiling = enable != 0;
  return LBM_OK;
}

int lbm_stream_probe(lbm_ctx *ctx, int n, double *ms_per_launch) {
  if (!ctx) return LBM_EINVAL;
  if (n < 2 || !ms_per_launch) return set_err(ctx, LBM_EINVAL, "need n >= 2 launches and an output");
  return dev_stream_probe(ctx, n, ms_per_launch);
}


int lbm_slot_map(const lbm_params *p, const uint8_t *mask, int parity, long long *read, long long *write) {
  std::string msg;
  if (!params_ok(p, msg)) return set_err(nullptr, LBM_EINVAL, msg);
  if (!read || !write || (parity != 0 && parity != 1))
    return set_err(nullptr, LBM_EINVAL, "need read and write arrays and parity 0 or 1");
  Geometry g;
  int rc = build_geometry(*p, mask, g, msg);
  if (rc != LBM_OK) return set_err(nullptr, rc, msg);
  KArgs k{};
  k.nx = p->nx;
  k.ny = p->ny;
  k.nz = p->nz;
  k.N = p->nx * p->ny * p->nz;
  for (int a = 0; a < 3; ++a) k.per[a] = p->periodic[a] ? 1 : 0;
  k.slip = p->slip;
  const uint8_t *fl = g.flags.data();
  const bool slip = p->slip != 0;
  if (p->lattice == LBM_D3Q19) {
    if (parity) slip ? slot_map_q<19, true, true>(k, fl, read, write) : slot_map_q<19, true, false>(k, fl, read, write);
    else slip ? slot_map_q<19, false, true>(k, fl, read, write) : slot_map_q<19, false, false>(k, fl, read, write);
  } else {
    if (parity) slip ? slot_map_q<27, true, true>(k, fl, read, write) : slot_map_q<27, true, false>(k, fl, read, write);
    else slip ? slot_map_q<27, false, true>(k, fl, read, write) : slot_map_q<27, false, false>(k, fl, read, write);
  }
  return LBM_OK;
}

int lbm_profile_read(lbm_ctx *ctx, double ms[3], long long count[3]) {
  if (!ctx || !ms || !count) return ctx ? set_err(ctx, LBM_EINVAL, "null output") : LBM_EINVAL;
  for (int k = 0; k < 3; ++k) {
    ms[k] = 0.0;
    count[k] = 0;
    if (!ctx->timers) continue;
    KernelTimer &t = ctx->timers[k];
    for (int s = 0; s < PROF_RING; ++s) drain_slot(t, s);
    ms[k] = t.ms;
    count[k] = t.count;
    t.ms = 0.0;
    t.count = 0;
  }
  return LBM_OK;
}

void lbm_free(lbm_ctx *ctx) {
  if (!ctx) return;
  if (ctx->timers) {
    for (int k = 0; k < 3; ++k)
      for (int s = 0; s < PROF_RING; ++s) {
        if (ctx->timers[k].start[s]) (void)hipEventDestroy(ctx->timers[k].start[s]);
        if (ctx->timers[k].stop[s]) (void)hipEventDestroy(ctx->timers[k].stop[s]);
      }
    delete[] ctx->timers;
  }
  delete ctx;
}

}  // extern "C"
