// Forward kernels of the wall-modeled LBM-LES step for gfx950 (wave64).
//
// One time step at parity p is two or three launches on the context's stream:
//   K1 k_wall_prepass  only for wall cells whose reference cell is itself a
//                      wall cell: friction velocity from the Spalding law
//                      (Sec. 2.2.1, Eq. (17)) by Newton in FP64 at the
//                      reference cell, modeled tangential velocity and strain;
//   K3 k_wall          one thread per wall cell: the same record for the
//                      other wall cells (their reference cells are bulk cells
//                      that no wall thread writes), then the sigma = 0
//                      reconstruction (equilibrium at the modeled velocity
//                      plus the non-equilibrium of Eq. (10) built from the
//                      wall-law strain) and the AA scatter;
//   K2 k_bulk          one thread per cell (128x2 tiles): AA gather, BGK
//                      collision with the Smagorinsky tau_eff (Eqs. (3),(4),
//                      (14)), homogenized velocity (Eq. (12)), Guo forcing,
//                      fringe/lid, AA scatter; skips wall cells.  It runs last
//                      because it writes the reference cells K1/K3 read.
// K2 and K3 touch disjoint slot sets (AA read set = write set per cell).
// The path is bound by HBM traffic: q loads and q stores per cell plus the
// flag byte, no contraction, so no MFMA.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "internal.h"
#include "lattice.h"
#include "wall.h"

namespace lbmk {

// Tile of one block (256 threads): rows of 128 cells, two wavefronts wide,
// two rows per block; or rows of 64 cells, four rows per block, when that
// leaves fewer lanes outside the domain (0 < nx mod 128 <= 64).  On odd steps
// the x-shifted accesses of a wavefront straddle cache lines; with the
// neighbouring wavefront of the same row in the same block, the partial lines
// are completed while still in L2.  Measured on K2: 128-wide tiles 1-2 %
// faster than 64-wide on the channel (nx 384) and the urban canopy (768);
// 64-wide 2 % faster on the 575^3 cavity, where 128-wide tiles leave 65 of
// 640 lanes per row idle; 256 x 1 loses on widths that are not multiples of
// 256.
constexpr int BLOCK = 256;

struct Tiles {
  unsigned nblocks;
  int gx, gy;
  int lx;  // log2 of the tile width (6 or 7)
};
static Tiles tiles_of(const KArgs &k) {
  Tiles t;
  const int r = k.nx % 128;
  t.lx = (r > 0 && r <= 64) ? 6 : 7;
  const int tw = 1 << t.lx, th = BLOCK >> t.lx;
  t.gx = (k.nx + tw - 1) / tw;
  t.gy = (k.ny + th - 1) / th;
  t.nblocks = (unsigned)t.gx * (unsigned)t.gy * (unsigned)k.nz;
  return t;
}

// Cell coordinates of this thread in the tiled grid; false when outside.
// rev = true walks the tiles in reverse order.  The bulk kernel reverses on
// odd steps, so each step starts where the previous one ended: the last
// tiles written are still partly held in the last-level (Infinity) cache
// and in L2 when the next step reads them.  On the 384x192x192 channel this
// raises the access pattern's rate by 3.7 % (a 764 MB state gains 8.7 %,
// a 6 GB one nothing).
__device__ __forceinline__ bool tile_xyz(const KArgs &k, Tiles t, unsigned block, int &x, int &y, int &z,
                                         bool rev = false) {
  unsigned L = xcd_remap(block, t.nblocks);
  if (rev) L = t.nblocks - 1u - L;
  const int tx = (int)(L % (unsigned)t.gx);
  const unsigned r = L / (unsigned)t.gx;
  const int ty = (int)(r % (unsigned)t.gy);
  z = (int)(r / (unsigned)t.gy);
  x = (tx << t.lx) + (int)(threadIdx.x & ((1u << t.lx) - 1u));
  y = ty * (BLOCK >> t.lx) + (int)(threadIdx.x >> t.lx);
  return x < k.nx && y < k.ny;
}

template <typename R>
__device__ __forceinline__ bool finite_pos(R v) {
  return v > R(0) && v < R(INFINITY);
}

// Deviation of the second-order equilibrium from the rest weight:
// f^eq_i(rho, v) - w_i = w_i [drho + rho (3 c.v + 9/2 (c.v)^2 - 3/2 v.v)].
template <typename R>
__device__ __forceinline__ R geq_dev(R w, R drho, R rho, R cv, R vv) {
  return w * (drho + rho * (R(3) * cv + R(4.5) * cv * cv - R(1.5) * vv));
}

// Fringe blend toward the inflow equilibrium and lid equilibrium (open
// boundary of the urban setup).
template <int Q, typename R>
__device__ __forceinline__ void fringe_blend(R g[Q], int x, int z, const KArgs &k) {
  if (x < k.fringe_start) return;
  const R lam = static_cast<const R *>(k.lam)[x];
  const R U = static_cast<const R *>(k.uin)[z];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R w = R(Lat<Q>::w(i));
    R cu = R(0);
    acc(cu, Lat<Q>::c(i, 0), U);
    const R ge = w * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * U * U);
    g[i] = (R(1) - lam) * g[i] + lam * ge;
  }
}

template <int Q, typename R>
__device__ __forceinline__ void lid_equilibrium(R g[Q], const KArgs &k) {
  const R U = R(k.u_lid);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R w = R(Lat<Q>::w(i));
    R cu = R(0);
    acc(cu, Lat<Q>::c(i, 0), U);
    g[i] = w * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * U * U);
  }
}


// Bulk collision on deviations g (sigma = 1): BGK with tau_eff from the
// non-equilibrium stress, homogenized velocity u_hat = phi u, Guo forcing.
// Opposite directions i and i+H share everything but a sign: with
//   f^eq_i - w = A + B, f^eq_ibar - w = A - B   (A even, B odd in c_i),
//   Guo_i = C + D,        Guo_ibar = C - D,
// the outputs are g*_i = c1 g_i + P + Qo and g*_ibar = c1 g_ibar + P - Qo.
// Returns false for a non-finite or non-positive density.
//
// RR = true: the recursive regularized collision (Sec. 2.2, Eqs. (6), (8),
// (9), (11), sigma = 1).  The equilibrium is third order and f - f^eq is
// replaced by f^(1) rebuilt from its Hermite coefficients: order 1,
// sum c (f - f^eq) = j - rho u = -F/2 (Guo velocity); order 2, Pi^neq; order 3,
// the recursion u_a Pi_bc + u_b Pi_ac + u_c Pi_ab.  The third-order terms are
// odd in c and join Qo; the outputs no longer carry c1 g_i.
//
// HYB = true (with RR): the hybrid of Eq. (7) with weight k.fdw = 1 - sigma
// of the finite-difference strain Sfd: the second-order part uses
// sigma Pi^neq - (1 - sigma) 2 rho c_s^2 tau S^FD, the third-order part keeps
// the factor sigma, the first-order part (-F/2) is kept whole.
template <int Q, typename R, bool POROUS, bool RR, bool HYB = false>
__device__ __forceinline__ bool collide_bulk(R g[Q], R phi, R smag, const KArgs &k, const R *Sfd = nullptr) {
  constexpr int H = Lat<Q>::H;
  // moments from pair sums s = g_i + g_ibar (even moments) and differences d = g_i - g_ibar (odd)
  R drho = g[0], jx = R(0), jy = R(0), jz = R(0);
  R mxx = R(0), myy = R(0), mzz = R(0), mxy = R(0), mxz = R(0), myz = R(0);
#pragma unroll
  for (int i = 1; i <= H; ++i) {
    const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
    const R sp = g[i] + g[i + H], dp = g[i] - g[i + H];
    drho += sp;
    acc(jx, cx, dp);
    acc(jy, cy, dp);
    acc(jz, cz, dp);
    acc(mxx, cx * cx, sp);
    acc(myy, cy * cy, sp);
    acc(mzz, cz * cz, sp);
    acc(mxy, cx * cy, sp);
    acc(mxz, cx * cz, sp);
    acc(myz, cy * cz, sp);
  }
  const R rho = R(1) + drho;
  const bool ok = finite_pos(rho);
  const R ir = R(1) / rho;
  const R Fx = R(k.F[0]), Fy = R(k.F[1]), Fz = R(k.F[2]);
  const R ux = (jx + R(0.5) * Fx) * ir, uy = (jy + R(0.5) * Fy) * ir, uz = (jz + R(0.5) * Fz) * ir;
  // Pi^neq = sum c c (f - f^eq(rho,u)) = M2(g) - drho c_s^2 I - rho u u
  const R cs2 = R(1.0 / 3.0);
  const R pxx = mxx - drho * cs2 - rho * ux * ux;
  const R pyy = myy - drho * cs2 - rho * uy * uy;
  const R pzz = mzz - drho * cs2 - rho * uz * uz;
  const R pxy = mxy - rho * ux * uy;
  const R pxz = mxz - rho * ux * uz;
  const R pyz = myz - rho * uy * uz;
  const R pn = sqrt(pxx * pxx + pyy * pyy + pzz * pzz + R(2) * (pxy * pxy + pxz * pxz + pyz * pyz));
  const R tau0 = R(k.tau0);
  const R tau = R(0.5) * (tau0 + sqrt(tau0 * tau0 + smag * pn * ir));
  const R om = R(1) / tau;
  const R c1 = R(1) - om, c2 = R(1) - R(0.5) * om;
  const R uu = ux * ux + uy * uy + uz * uz;
  const R vx = POROUS ? phi * ux : ux, vy = POROUS ? phi * uy : uy, vz = POROUS ? phi * uz : uz;
  const R vv = vx * vx + vy * vy + vz * vz;
  const R uF = ux * Fx + uy * Fy + uz * Fz;
  if constexpr (RR) {
    // third-order coefficients of f^eq(rho, v) + c1 f^(1): A = rho v v v + c1 sigma A1
    R A[7], A1[7], K[7];
    cube_tensor(rho, vx, vy, vz, A);
    R sig = R(1);
    R hxx = pxx, hyy = pyy, hzz = pzz, hxy = pxy, hxz = pxz, hyz = pyz;  // second-order coefficient
    if constexpr (HYB) {
      const R fw = R(k.fdw);
      sig = R(1) - fw;
      const R fs = fw * R(2.0 / 3.0) * rho * tau;  // (1 - sigma) 2 rho c_s^2 tau
      hxx = sig * pxx - fs * Sfd[0];
      hyy = sig * pyy - fs * Sfd[1];
      hzz = sig * pzz - fs * Sfd[2];
      hxy = sig * pxy - fs * Sfd[3];
      hxz = sig * pxz - fs * Sfd[4];
      hyz = sig * pyz - fs * Sfd[5];
    }
    A1[0] = R(2) * ux * pxy + uy * pxx;
    A1[1] = R(2) * ux * pxz + uz * pxx;
    A1[2] = R(2) * uy * pxy + ux * pyy;
    A1[3] = R(2) * uy * pyz + uz * pyy;
    A1[4] = R(2) * uz * pxz + ux * pzz;
    A1[5] = R(2) * uz * pyz + uy * pzz;
    A1[6] = ux * pyz + uy * pxz + uz * pxy;
    const R c1s = c1 * sig;
#pragma unroll
    for (int m = 0; m < 7; ++m) A[m] += c1s * A1[m];
    third_coefs<Q, R>(A, K);
    const R tr3 = (hxx + hyy + hzz) * cs2;
    // rest: f^eq - w = w0 (drho - 3/2 rho v.v); f^(1)_0 = -9/2 w0 c_s^2 tr Pi; Guo -3 w0 u.F
    {
      const R w = R(Lat<Q>::w(0));
      g[0] = w * (drho - R(1.5) * rho * vv) - c1 * R(4.5) * w * tr3 + c2 * (R(-3) * w * uF);
    }
#pragma unroll
    for (int i = 1; i <= H; ++i) {
      const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
      const R w = R(Lat<Q>::w(i));
      const R cu = dot3(cx, cy, cz, ux, uy, uz);
      const R cv = POROUS ? dot3(cx, cy, cz, vx, vy, vz) : cu;
      const R cF = dot3(cx, cy, cz, Fx, Fy, Fz);
      R cPc = R(0);  // c . Pi . c (of the second-order coefficient)
      acc(cPc, cx * cx, hxx);
      acc(cPc, cy * cy, hyy);
      acc(cPc, cz * cz, hzz);
      acc(cPc, cx * cy, R(2) * hxy);
      acc(cPc, cx * cz, R(2) * hxz);
      acc(cPc, cy * cz, R(2) * hyz);
      const R P = w * (drho + rho * (R(4.5) * cv * cv - R(1.5) * vv) + c1 * R(4.5) * (cPc - tr3) +
                       c2 * (R(9) * cu * cF - R(3) * uF));
      // odd part: 3 w rho c.v + w sum_k P_k K_k + c1 (3 w c.a1, a1 = -F/2) + c2 3 w c.F
      const R Qo = w * (R(3) * rho * cv + third_term<Q, R>(i, K) + (R(3) * c2 - R(1.5) * c1) * cF);
      g[i] = P + Qo;
      g[i + H] = P - Qo;
    }
    return ok;
  }
  // rest population: A = w0 (drho - 3/2 rho v.v), B = C - (-3 w0 u.F) = D = 0
  {
    const R w = R(Lat<Q>::w(0));
    const R au = w * (drho - R(1.5) * rho * uu);
    const R av = POROUS ? w * (drho - R(1.5) * rho * vv) : au;
    g[0] = c1 * g[0] + (av - c1 * au) + c2 * (R(-3) * w * uF);
  }
#pragma unroll
  for (int i = 1; i <= H; ++i) {
    const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
    const R w = R(Lat<Q>::w(i));
    const R cu = dot3(cx, cy, cz, ux, uy, uz);
    const R cF = dot3(cx, cy, cz, Fx, Fy, Fz);
    const R Au = w * (drho + rho * (R(4.5) * cu * cu - R(1.5) * uu));
    const R Bu = R(3) * w * rho * cu;
    R Av = Au, Bv = Bu;
    if (POROUS) {
      const R cv = dot3(cx, cy, cz, vx, vy, vz);
      Av = w * (drho + rho * (R(4.5) * cv * cv - R(1.5) * vv));
      Bv = R(3) * w * rho * cv;
    }
    const R C = w * (R(9) * cu * cF - R(3) * uF);
    const R D = R(3) * w * cF;
    const R P = (Av - c1 * Au) + c2 * C;
    const R Qo = (Bv - c1 * Bu) + c2 * D;
    const R gi = g[i], gj = g[i + H];
    g[i] = c1 * gi + P + Qo;
    g[i + H] = c1 * gj + P - Qo;
  }
  return ok;
}

// ---------------------------------------------------------------------------
// Open x faces (Sec. 2.2.2: regularized local velocity inlet; Sec. 3.2: fixed
// local pressure outlet).  The pre-collision deviations g of an inlet
// (x = 0) or outlet (x = nx - 1) cell are rebuilt in place:
//  - with n the outward normal (-x at the inlet, +x at the outlet), the
//    populations with c.n < 0 enter through the face and are unknown;
//  - rho (1 + u.n) = s_0 + 2 s_+, where s_0 sums the populations with c.n = 0
//    and s_+ those with c.n > 0 (in deviations: 1 + G_0 + 2 G_+, since their
//    weights sum to 2/3 and 1/6);
//  - inlet: u from the inlet velocity field (u_in(z) along x plus the vortex
//    method's in-plane part, k_inflow), rho from that relation; outlet:
//    rho = rho_out, u.n from it, no tangential velocity;
//  - inlet (regularized): the non-equilibrium h = g - g^eq of an unknown
//    population is that of its opposite, Pi = sum c c h, and
//    g = g^eq + 9/2 w (c.Pi.c - tr Pi/3);
//  - outlet: g = g^eq.  A non-equilibrium rebuilt there from the arriving
//    populations feeds the over-relaxed (tau near 1/2) non-equilibrium back
//    through the face: perturbations then grow without bound at small
//    viscosity, while the equilibrium outlet keeps them at their size.
// With the recursive regularized model the equilibrium is third order (for a
// velocity along x, as at the outlet, its third-order terms vanish: the
// lattices carry no xxx component).
// ---------------------------------------------------------------------------
template <int Q, typename R, bool RR>
__device__ __forceinline__ void open_rebuild(R g[Q], bool outlet, int y, int z, const KArgs &k) {
  constexpr int H = (Q - 1) / 2;
  const int nxo = outlet ? 1 : -1;  // x component of the outward normal
  R gpar = g[0], gout = R(0);
#pragma unroll
  for (int i = 1; i <= H; ++i) {
    const int cx = Lat<Q>::c(i, 0);
    if (cx == 0) {
      gpar += g[i] + g[i + H];
    } else {
      gout += cx * nxo > 0 ? g[i] : g[i + H];  // the member of the pair that leaves through the face
    }
  }
  const R m = gpar + R(2) * gout;  // s_0 + 2 s_+ - 1
  R drho, rho, ux, uy = R(0), uz = R(0);
  if (outlet) {
    drho = R(k.rho_out - 1.0);
    rho = R(1) + drho;
    ux = (m - drho) / rho;  // u.n with n = +x
  } else {
    // inlet velocity field: the mean profile plus the vortex method's in-plane part
    const R *f = static_cast<const R *>(k.inflow);
    const int face = k.ny * k.nz, c2 = y + k.ny * z;
    ux = f[c2];
    uy = f[face + c2];
    uz = f[2 * face + c2];
    const R un = -ux;
    drho = (m - un) / (R(1) + un);
    rho = R(1) + drho;
  }
  const R uu = ux * ux + uy * uy + uz * uz;
  // equilibrium deviations, third order with the recursive regularized model
  R K[7];
  if constexpr (RR) {
    R A[7];
    cube_tensor(rho, ux, uy, uz, A);
    third_coefs<Q, R>(A, K);
  }
  R geq[Q];
  geq[0] = R(Lat<Q>::w(0)) * (drho - R(1.5) * rho * uu);
#pragma unroll
  for (int i = 1; i <= H; ++i) {
    const R w = R(Lat<Q>::w(i));
    const R cu = dot3(Lat<Q>::c(i, 0), Lat<Q>::c(i, 1), Lat<Q>::c(i, 2), ux, uy, uz);
    const R P = w * (drho + rho * (R(4.5) * cu * cu - R(1.5) * uu));
    R Qo = w * R(3) * rho * cu;
    if constexpr (RR) Qo += w * third_term<Q, R>(i, K);
    geq[i] = P + Qo;
    geq[i + H] = P - Qo;
  }
  if (outlet) {
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = geq[i];
    return;
  }
  R pxx = R(0), pyy = R(0), pzz = R(0), pxy = R(0), pxz = R(0), pyz = R(0);
#pragma unroll
  for (int i = 1; i <= H; ++i) {
    const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
    R hs;  // h_i + h_ibar
    if (cx == 0) {
      hs = (g[i] - geq[i]) + (g[i + H] - geq[i + H]);
    } else {
      const int kn = cx * nxo > 0 ? i : i + H;  // the known member of the pair
      hs = R(2) * (g[kn] - geq[kn]);
    }
    acc(pxx, cx * cx, hs);
    acc(pyy, cy * cy, hs);
    acc(pzz, cz * cz, hs);
    acc(pxy, cx * cy, hs);
    acc(pxz, cx * cz, hs);
    acc(pyz, cy * cz, hs);
  }
  const R tr3 = (pxx + pyy + pzz) * R(1.0 / 3.0);
  g[0] = geq[0] - R(4.5) * R(Lat<Q>::w(0)) * tr3;
#pragma unroll
  for (int i = 1; i <= H; ++i) {
    const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
    R cPc = R(0);
    acc(cPc, cx * cx, pxx);
    acc(cPc, cy * cy, pyy);
    acc(cPc, cz * cz, pzz);
    acc(cPc, cx * cy, R(2) * pxy);
    acc(cPc, cx * cz, R(2) * pxz);
    acc(cPc, cy * cz, R(2) * pyz);
    const R r = R(4.5) * R(Lat<Q>::w(i)) * (cPc - tr3);
    g[i] = geq[i] + r;
    g[i + H] = geq[i + H] + r;
  }
}

// Inlet velocity field, one thread per cell (y, z) of the inflow plane: the
// mean profile u_in(z) along x plus the vortex method's in-plane velocity of
// nvort vortices (y_i, z_i, Gamma_i) at the cell centre (Sec. 2.2.2):
// u_vortex = 1/(2 pi) sum_i Gamma_i ((p_i - x) x d)(1 - exp(-r^2/(2 sigma^2)))/r^2
// with d = +x, i.e. (0, Delta z, -Delta y) for Delta = p_i - x.  Summed in FP64.
template <typename R>
__global__ __launch_bounds__(256) void k_inflow(R *__restrict__ field, const double *__restrict__ vort, int nvort,
                                                double sigma, KArgs k) {
  const int face = k.ny * k.nz;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= face) return;
  const int y = t % k.ny, z = t / k.ny;
  const double yc = y + 0.5, zc = z + 0.5;
  const double inv2s2 = 1.0 / (2.0 * sigma * sigma), inv2pi = 1.0 / (2.0 * 3.14159265358979323846);
  double uy = 0.0, uz = 0.0;
  for (int i = 0; i < nvort; ++i) {
    const double dy = vort[3 * i] - yc, dz = vort[3 * i + 1] - zc;
    const double r2 = dy * dy + dz * dz;
    if (r2 == 0.0) continue;
    const double f = vort[3 * i + 2] * inv2pi * (1.0 - exp(-r2 * inv2s2)) / r2;
    uy += f * dz;
    uz -= f * dy;
  }
  field[t] = static_cast<const R *>(k.uin)[z];
  field[face + t] = R(uy);
  field[2 * face + t] = R(uz);
}

// ---------------------------------------------------------------------------
// K2: fused gather / collide / scatter over all non-wall fluid cells.
// ---------------------------------------------------------------------------
// Gather, collide, scatter of one cell.  With LINKS = false the cell has no
// solid link and every slot is the plain AA one (32-bit offsets from a
// per-direction base); with LINKS = true slots follow the bounce-back map.
template <int Q, typename S, bool ODD, bool POROUS, bool LINKS, bool RR, bool HYB, bool OPEN, bool SLIP = false>
__device__ __forceinline__ void bulk_cell(S *__restrict__ pop, const typename Store<S>::R *__restrict__ phi,
                                          const uint8_t *__restrict__ flags, const KArgs &k, const Nb &n,
                                          LinkMask sm, uint8_t fl, int x, int y, int z,
                                          int *__restrict__ errflag) {
  using R = typename Store<S>::R;
  const size_t N = (size_t)k.N;
  R g[Q];
  if (fl & FL_LID) {
    lid_equilibrium<Q, R>(g, k);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (LINKS) {
        g[i] = Store<S>::ld(pop + read_slot<Q, ODD, SLIP>(n, sm, i, N));
      } else {
        int dir;
        const int idx = plain_read<Q, ODD>(n, i, dir);
        g[i] = Store<S>::ld(slot_at(pop, dir, N, idx));
      }
    }
    if constexpr (OPEN) {
      if (fl & (FL_INLET | FL_OUTLET)) open_rebuild<Q, R, RR>(g, (fl & FL_OUTLET) != 0, y, z, k);
    }
    const R ph = POROUS ? phi[n.cell] : R(1);
    R Sfd[6];
    if constexpr (HYB) fd_strain<R>(n, k, Sfd);
    if (!collide_bulk<Q, R, POROUS, RR, HYB>(g, ph, smag_of<R>(k, n.cell), k, Sfd)) atomicOr(errflag, 1);
  }
  // the outlet plane is left out of the fringe
  if (!OPEN || !(fl & FL_OUTLET)) fringe_blend<Q, R>(g, x, z, k);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (LINKS) {
      Store<S>::st(pop + write_slot<Q, ODD, SLIP>(n, sm, i, N), g[i]);
    } else {
      int dir;
      const int idx = plain_write<Q, ODD>(n, i, dir);
      Store<S>::st(slot_at(pop, dir, N, idx), g[i]);
    }
  }
}

template <int Q, typename S, bool ODD, bool POROUS, int SOLID, bool RR, bool HYB, bool OPEN = false>
__global__ __launch_bounds__(BLOCK) void k_bulk(S *__restrict__ pop, const uint8_t *__restrict__ flags,
                                                const typename Store<S>::R *__restrict__ phi, KArgs k,
                                                Tiles t, int *__restrict__ errflag) {
  int x, y, z;
  if (!tile_xyz(k, t, blockIdx.x, x, y, z, ODD)) return;
  const Nb n = make_nb(x, y, z, k);
  const uint8_t fl = flags[n.cell];
  // wall cells have a kernel of their own; OPEN: the cells of the inlet and
  // outlet planes are updated here, in the rows whose cache lines they share
  if (!(fl & FL_FLUID) || (fl & FL_WALL)) return;
  LinkMask sm = 0;
  if (SOLID && ODD && (fl & FL_NEAR)) sm = solid_mask<Q, SOLID == 2>(n, flags);
  // cells without solid links (all but a thin layer) take the plain-address path
  if (SOLID && ODD && sm != 0u)
    bulk_cell<Q, S, ODD, POROUS, true, RR, HYB, OPEN, SOLID == 2>(pop, phi, flags, k, n, sm, fl, x, y, z, errflag);
  else
    bulk_cell<Q, S, ODD, POROUS, false, RR, HYB, OPEN>(pop, phi, flags, k, n, sm, fl, x, y, z, errflag);
}

// ---------------------------------------------------------------------------
// Memory-system ceiling of the bulk kernel's accesses: the same tiles, block
// order, cell selection and slot map, no collision.  Every cell the bulk
// kernel updates loads its q slots and stores each value back to the slot it
// came from, so the state is unchanged.  The stores go through an empty asm
// that hides the value from the compiler (a store of a just-loaded value to
// its own address would otherwise be removed).
// ---------------------------------------------------------------------------
template <typename S>
struct Bits;
template <>
struct Bits<double> {
  using T = uint64_t;
};
template <>
struct Bits<float> {
  using T = uint32_t;
};
template <>
struct Bits<_Float16> {
  using T = uint16_t;
};
template <typename U>
__device__ __forceinline__ void opaque(U &v) {
  if constexpr (sizeof(U) == 2) {
    uint32_t t = v;
    asm volatile("" : "+v"(t));
    v = (U)t;
  } else {
    asm volatile("" : "+v"(v));
  }
}
template <int Q, typename S, bool ODD, int SOLID>
__global__ __launch_bounds__(BLOCK) void k_stream_probe(S *__restrict__ pop_, const uint8_t *__restrict__ flags,
                                                        KArgs k, Tiles t) {
  using U = typename Bits<S>::T;
  U *pop = reinterpret_cast<U *>(pop_);
  int x, y, z;
  if (!tile_xyz(k, t, blockIdx.x, x, y, z, ODD)) return;
  const Nb n = make_nb(x, y, z, k);
  const uint8_t fl = flags[n.cell];
  if (!(fl & FL_FLUID) || (fl & FL_WALL)) return;
  LinkMask sm = 0;
  if (SOLID && ODD && (fl & FL_NEAR)) sm = solid_mask<Q, SOLID == 2>(n, flags);
  const size_t N = (size_t)k.N;
  U v[Q];
  if (SOLID && ODD && sm != 0u) {
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = pop[read_slot<Q, ODD, SOLID == 2>(n, sm, i, N)];
#pragma unroll
    for (int i = 0; i < Q; ++i) opaque(v[i]);
#pragma unroll
    for (int i = 0; i < Q; ++i) pop[read_slot<Q, ODD, SOLID == 2>(n, sm, i, N)] = v[i];
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      int dir;
      const int idx = plain_read<Q, ODD>(n, i, dir);
      v[i] = *slot_at(pop, dir, N, idx);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) opaque(v[i]);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      int dir;
      const int idx = plain_read<Q, ODD>(n, i, dir);
      *slot_at(pop, dir, N, idx) = v[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Wall record of wall cell w (reference cell r, wall cell b): reads the
// reference cell's current populations and writes t, u_tau u+_b, G, tau_eff
// (the computation itself is wall_record_of in wall.h).
// ---------------------------------------------------------------------------
template <int Q, typename S, bool ODD, bool SLIP>
__device__ __forceinline__ void wall_record(const S *__restrict__ pop, const uint64_t *__restrict__ wmask, int w,
                                            int b, int r, double *__restrict__ rec, int nwall, const KArgs &k,
                                            int *__restrict__ errflag) {
  double rho, u[3];
  ref_velocity<Q, S, ODD, SLIP>(pop, wmask[(size_t)nwall + w], r, k, rho, u);
  const size_t M = (size_t)nwall;
  const double n[3] = {rec[WR_NX * M + w], rec[WR_NY * M + w], rec[WR_NZ * M + w]};
  const WallRec wr =
      wall_record_of(u, n, rec[WR_YR * M + w], rec[WR_YB * M + w], r == b, cs2_of<typename Store<S>::R>(k, b), k);
  if (wr.fail) atomicOr(errflag, 2);
  rec[WR_TX * M + w] = wr.t[0];
  rec[WR_TY * M + w] = wr.t[1];
  rec[WR_TZ * M + w] = wr.t[2];
  rec[WR_UTAN * M + w] = wr.utan;
  rec[WR_G * M + w] = wr.G;
  rec[WR_TAU * M + w] = wr.tau;
  rec[WR_UTAU * M + w] = wr.utau;
}

template <int Q, typename S, bool ODD, bool SLIP>
__global__ __launch_bounds__(256) void k_wall_prepass(const S *__restrict__ pop, const uint64_t *__restrict__ wmask,
                                                      const int *__restrict__ wcell, const int *__restrict__ wref,
                                                      const int *__restrict__ list, int nlist,
                                                      double *__restrict__ rec, int nwall, KArgs k,
                                                      int *__restrict__ errflag) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nlist) return;
  const int w = list[j];
  wall_record<Q, S, ODD, SLIP>(pop, wmask, w, wcell[w], wref[w], rec, nwall, k, errflag);
}

// ---------------------------------------------------------------------------
// K3: wall reconstruction (sigma = 0, solid velocity = modeled velocity).
// ---------------------------------------------------------------------------
template <int Q, typename S, bool ODD, bool SLIP>
__global__ __launch_bounds__(256) void k_wall(S *__restrict__ pop, const uint64_t *__restrict__ wmask,
                                              const int *__restrict__ wcell, const int *__restrict__ wref,
                                              const uint8_t *__restrict__ refwall, double *__restrict__ rec,
                                              int nwall, KArgs k, int *__restrict__ errflag) {
  using R = typename Store<S>::R;
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwall) return;
  const int b = wcell[w];
  int x, y, z;
  cell_xyz(b, k, x, y, z);
  const Nb n = make_nb(x, y, z, k);
  // the cell's link mask, precomputed from the static geometry
  const LinkMask sm = ODD ? wmask[w] : 0u;
  const size_t N = (size_t)k.N;
  R g[Q];
  R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    g[i] = Store<S>::ld(pop + read_slot<Q, ODD, SLIP>(n, sm, i, N));
    drho += g[i];
    acc(jx, Lat<Q>::c(i, 0), g[i]);
    acc(jy, Lat<Q>::c(i, 1), g[i]);
    acc(jz, Lat<Q>::c(i, 2), g[i]);
  }
  // The record of a wall cell whose reference is not a wall cell is computed
  // here (no other thread of this launch writes that reference); the others
  // were computed by k_wall_prepass before this launch.  It comes after the
  // loads above, so that their latency overlaps the Newton solves.
  if (!refwall[w]) wall_record<Q, S, ODD, SLIP>(pop, wmask, w, b, wref[w], rec, nwall, k, errflag);
  const R rho = R(1) + drho;
  if (!finite_pos(rho)) atomicOr(errflag, 1);
  const R Fx = R(k.F[0]), Fy = R(k.F[1]), Fz = R(k.F[2]);
  const R ir = R(1) / rho;
  const R ux = (jx + R(0.5) * Fx) * ir, uy = (jy + R(0.5) * Fy) * ir, uz = (jz + R(0.5) * Fz) * ir;
  const size_t M = (size_t)nwall;
  const R nx = R(rec[WR_NX * M + w]), ny = R(rec[WR_NY * M + w]), nz = R(rec[WR_NZ * M + w]);
  const R tx = R(rec[WR_TX * M + w]), ty = R(rec[WR_TY * M + w]), tz = R(rec[WR_TZ * M + w]);
  const R utan = R(rec[WR_UTAN * M + w]), G = R(rec[WR_G * M + w]), tau = R(rec[WR_TAU * M + w]);
  const R un = ux * nx + uy * ny + uz * nz;
  const R vx = utan * tx + un * nx, vy = utan * ty + un * ny, vz = utan * tz + un * nz;
  const R vv = vx * vx + vy * vy + vz * vz;
  const R vF = vx * Fx + vy * Fy + vz * Fz;
  const R om = R(1) / tau;
  const R c1 = R(1) - om, c2 = R(1) - R(0.5) * om;
  const R fd = R(-3) * rho * tau * G;  // f^(1,FD)_i = fd * w_i (c.t)(c.n)
  // hybrid collision (sigma = 0 in the wall region): the full finite-difference
  // strain whose wall-normal shear s = S n - (n.S.n) n (every tangential
  // direction) is replaced by the wall law's, G/2 along t:
  // S' = S + (e n^T + n e^T), e = (G/2) t - s; then
  // f^(1,FD)_i = -3 w_i rho tau (c.S'.c - c_s^2 tr S')
  R Sw[6] = {};
  const bool full = k.fdw > 0.0;
  if (full) {
    fd_strain<R>(n, k, Sw);
    const R snx = Sw[0] * nx + Sw[3] * ny + Sw[4] * nz;
    const R sny = Sw[3] * nx + Sw[1] * ny + Sw[5] * nz;
    const R snz = Sw[4] * nx + Sw[5] * ny + Sw[2] * nz;
    const R nSn = nx * snx + ny * sny + nz * snz;
    const R hg = R(0.5) * G;
    const R ex = hg * tx - (snx - nSn * nx), ey = hg * ty - (sny - nSn * ny), ez = hg * tz - (snz - nSn * nz);
    Sw[0] += R(2) * ex * nx;
    Sw[1] += R(2) * ey * ny;
    Sw[2] += R(2) * ez * nz;
    Sw[3] += ex * ny + nx * ey;
    Sw[4] += ex * nz + nx * ez;
    Sw[5] += ey * nz + ny * ez;
  }
  const R trw = (Sw[0] + Sw[1] + Sw[2]) * R(1.0 / 3.0);
  // recursive regularized model: third-order equilibrium at the modeled velocity
  R K[7] = {};
  if (k.rr) {
    R A[7];
    cube_tensor(rho, vx, vy, vz, A);
    third_coefs<Q, R>(A, K);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
    const R w = R(Lat<Q>::w(i));
    const R cv = dot3(cx, cy, cz, vx, vy, vz);
    const R ct = dot3(cx, cy, cz, tx, ty, tz);
    const R cn = dot3(cx, cy, cz, nx, ny, nz);
    const R cF = dot3(cx, cy, cz, Fx, Fy, Fz);
    const R ge = geq_dev(w, drho, rho, cv, vv);
    R ffd;
    if (full) {
      R cSc = R(0);
      acc(cSc, cx * cx, Sw[0]);
      acc(cSc, cy * cy, Sw[1]);
      acc(cSc, cz * cz, Sw[2]);
      acc(cSc, cx * cy, R(2) * Sw[3]);
      acc(cSc, cx * cz, R(2) * Sw[4]);
      acc(cSc, cy * cz, R(2) * Sw[5]);
      ffd = R(-3) * w * rho * tau * (cSc - trw);
    } else {
      ffd = fd * w * ct * cn;
    }
    const R guo = w * (R(3) * (cF - vF) + R(9) * cv * cF);
    g[i] = ge + c1 * ffd + c2 * guo;
    if (k.rr) g[i] += w * third_term<Q, R>(i, K);
  }
  fringe_blend<Q, R>(g, x, z, k);
#pragma unroll
  for (int i = 0; i < Q; ++i) Store<S>::st(pop + write_slot<Q, ODD, SLIP>(n, sm, i, N), g[i]);
}

// ---------------------------------------------------------------------------
// K0: initial equilibrium; moments; natural-order export / import.
// ---------------------------------------------------------------------------
template <int Q, typename S>
__global__ __launch_bounds__(BLOCK) void k_init_eq(S *__restrict__ pop, const uint8_t *__restrict__ flags,
                                                   const double *__restrict__ rho0, const double *__restrict__ u0,
                                                   KArgs k, Tiles t) {
  int x, y, z;
  if (!tile_xyz(k, t, blockIdx.x, x, y, z)) return;
  const int c = x + k.nx * (y + k.ny * z);
  const size_t N = (size_t)k.N;
  if (!(flags[c] & FL_FLUID)) {
#pragma unroll
    for (int i = 0; i < Q; ++i) Store<S>::st(pop + (size_t)i * N + c, typename Store<S>::R(0));
    return;
  }
  const double rho = rho0 ? rho0[c] : 1.0;
  const double drho = rho0 ? rho0[c] - 1.0 : 0.0;
  const double ux = u0 ? u0[c] : 0.0, uy = u0 ? u0[N + c] : 0.0, uz = u0 ? u0[2 * N + c] : 0.0;
  const double uu = ux * ux + uy * uy + uz * uz;
  double K[7] = {};
  if (k.rr) {  // third-order equilibrium
    double A[7];
    cube_tensor(rho, ux, uy, uz, A);
    third_coefs<Q, double>(A, K);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double cu = dot3(Lat<Q>::c(i, 0), Lat<Q>::c(i, 1), Lat<Q>::c(i, 2), ux, uy, uz);
    double gi = geq_dev(Lat<Q>::w(i), drho, rho, cu, uu);
    if (k.rr) gi += Lat<Q>::w(i) * third_term<Q, double>(i, K);
    Store<S>::st(pop + (size_t)i * N + c, (typename Store<S>::R)gi);
  }
}

template <int Q, typename S, bool ODD, int SOLID>
__device__ __forceinline__ bool gather_state(const S *__restrict__ pop, const uint8_t *__restrict__ flags,
                                             const KArgs &k, int x, int y, int z, Nb &n,
                                             typename Store<S>::R g[Q]) {
  n = make_nb(x, y, z, k);
  const uint8_t fl = flags[n.cell];
  if (!(fl & FL_FLUID)) return false;
  LinkMask sm = 0;
  if (SOLID && ODD && (fl & FL_NEAR)) sm = solid_mask<Q, SOLID == 2>(n, flags);
#pragma unroll
  for (int i = 0; i < Q; ++i) g[i] = Store<S>::ld(pop + read_slot<Q, ODD, SOLID == 2>(n, sm, i, (size_t)k.N));
  return true;
}

// The hybrid's velocity field: (Guo velocity, rho) at fluid cells, 0 elsewhere.
template <int Q, typename S, bool ODD, int SOLID>
__global__ __launch_bounds__(BLOCK) void k_velocity4(const S *__restrict__ pop, const uint8_t *__restrict__ flags,
                                                     V4<typename Store<S>::R> *__restrict__ out, KArgs k, Tiles t) {
  using R = typename Store<S>::R;
  int x, y, z;
  if (!tile_xyz(k, t, blockIdx.x, x, y, z)) return;
  Nb n;
  R g[Q];
  if (!gather_state<Q, S, ODD, SOLID>(pop, flags, k, x, y, z, n, g)) {
    out[x + k.nx * (y + k.ny * z)] = V4<R>{R(0), R(0), R(0), R(0)};
    return;
  }
  R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += g[i];
    acc(jx, Lat<Q>::c(i, 0), g[i]);
    acc(jy, Lat<Q>::c(i, 1), g[i]);
    acc(jz, Lat<Q>::c(i, 2), g[i]);
  }
  const R rho = R(1) + drho;
  out[n.cell] = V4<R>{(jx + R(0.5) * R(k.F[0])) / rho, (jy + R(0.5) * R(k.F[1])) / rho,
                      (jz + R(0.5) * R(k.F[2])) / rho, rho};
}

template <int Q, typename S, bool ODD, int SOLID>
__global__ __launch_bounds__(BLOCK) void k_moments(const S *__restrict__ pop, const uint8_t *__restrict__ flags,
                                                   typename Store<S>::R *__restrict__ rho_out,
                                                   typename Store<S>::R *__restrict__ u_out, KArgs k, Tiles t) {
  using R = typename Store<S>::R;
  int x, y, z;
  if (!tile_xyz(k, t, blockIdx.x, x, y, z)) return;
  Nb n;
  R g[Q];
  const size_t N = (size_t)k.N;
  if (!gather_state<Q, S, ODD, SOLID>(pop, flags, k, x, y, z, n, g)) {
    const int c = x + k.nx * (y + k.ny * z);
    if (rho_out) rho_out[c] = R(0);
    if (u_out) u_out[c] = u_out[N + c] = u_out[2 * N + c] = R(0);
    return;
  }
  R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += g[i];
    acc(jx, Lat<Q>::c(i, 0), g[i]);
    acc(jy, Lat<Q>::c(i, 1), g[i]);
    acc(jz, Lat<Q>::c(i, 2), g[i]);
  }
  const R rho = R(1) + drho;
  if (rho_out) rho_out[n.cell] = rho;
  if (u_out) {
    u_out[n.cell] = (jx + R(0.5) * R(k.F[0])) / rho;
    u_out[N + n.cell] = (jy + R(0.5) * R(k.F[1])) / rho;
    u_out[2 * N + n.cell] = (jz + R(0.5) * R(k.F[2])) / rho;
  }
}

template <int Q, typename S, bool ODD, int SOLID>
__global__ __launch_bounds__(BLOCK) void k_export(const S *__restrict__ pop, const uint8_t *__restrict__ flags,
                                                  typename Store<S>::R *__restrict__ f, KArgs k, Tiles t) {
  using R = typename Store<S>::R;
  int x, y, z;
  if (!tile_xyz(k, t, blockIdx.x, x, y, z)) return;
  Nb n;
  R g[Q];
  const size_t N = (size_t)k.N;
  const bool fluid = gather_state<Q, S, ODD, SOLID>(pop, flags, k, x, y, z, n, g);
#pragma unroll
  for (int i = 0; i < Q; ++i) f[(size_t)i * N + n.cell] = fluid ? R(Lat<Q>::w(i)) + g[i] : R(0);
}

template <int Q, typename S, bool ODD, int SOLID>
__global__ __launch_bounds__(BLOCK) void k_import(S *__restrict__ pop, const uint8_t *__restrict__ flags,
                                                  const typename Store<S>::R *__restrict__ f, KArgs k, Tiles t) {
  using R = typename Store<S>::R;
  int x, y, z;
  if (!tile_xyz(k, t, blockIdx.x, x, y, z)) return;
  const Nb n = make_nb(x, y, z, k);
  const uint8_t fl = flags[n.cell];
  if (!(fl & FL_FLUID)) return;
  LinkMask sm = 0;
  if (SOLID && ODD && (fl & FL_NEAR)) sm = solid_mask<Q, SOLID == 2>(n, flags);
  const size_t N = (size_t)k.N;
#pragma unroll
  for (int i = 0; i < Q; ++i)
    Store<S>::st(pop + read_slot<Q, ODD, SOLID == 2>(n, sm, i, N), f[(size_t)i * N + n.cell] - R(Lat<Q>::w(i)));
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions: wave64 shuffle tree, LDS across the block's
// four waves, one partial per block, then a single-block finalise in fixed
// order.  Grid-stride over tiles with a fixed grid, so the summation order
// depends only on the domain size.
// ---------------------------------------------------------------------------
constexpr int RED_BLOCKS = 1024;
constexpr int NRED = 8;
// partials of RED_BLOCKS blocks, then NRED finalised sums
constexpr int SCRATCH_DOUBLES = RED_BLOCKS * NRED + NRED;
constexpr int MAX_DEVICES = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double *__restrict__ out) {
  __shared__ double sh[BLOCK / 64][NRED];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < NV; ++a) v[a] = wave_sum(v[a]);
  if (lane == 0)
#pragma unroll
    for (int a = 0; a < NV; ++a) sh[wv][a] = v[a];
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int q = 0; q < BLOCK / 64; ++q) s += sh[q][threadIdx.x];
    out[(size_t)blockIdx.x * NRED + threadIdx.x] = s;
  }
}

// mode 0: {sum drho, sum jx, sum jy, sum jz, fluid cells} over fluid cells.
// mode 1: {sum rho at x = p0, sum rho at x = p1, sum rho|u|^2/2, cells at
//          x = p0, cells at x = p1, fluid cells}.
template <int Q, typename S, bool ODD, int SOLID>
__global__ __launch_bounds__(BLOCK) void k_reduce(const S *__restrict__ pop, const uint8_t *__restrict__ flags,
                                                  KArgs k, Tiles t, int mode, int p0, int p1,
                                                  double *__restrict__ partial) {
  using R = typename Store<S>::R;
  double v[NRED] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (unsigned b = blockIdx.x; b < t.nblocks; b += gridDim.x) {
    int x, y, z;
    if (!tile_xyz(k, t, b, x, y, z)) continue;
    Nb n;
    R g[Q];
    if (!gather_state<Q, S, ODD, SOLID>(pop, flags, k, x, y, z, n, g)) continue;
    double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double gi = (double)g[i];
      drho += gi;
      acc(jx, Lat<Q>::c(i, 0), gi);
      acc(jy, Lat<Q>::c(i, 1), gi);
      acc(jz, Lat<Q>::c(i, 2), gi);
    }
    if (mode == 0) {
      v[0] += drho;
      v[1] += jx;
      v[2] += jy;
      v[3] += jz;
      v[4] += 1.0;
    } else {
      const double rho = 1.0 + drho;
      const double mx = jx + 0.5 * k.F[0], my = jy + 0.5 * k.F[1], mz = jz + 0.5 * k.F[2];
      if (x == p0) {
        v[0] += rho;
        v[3] += 1.0;
      }
      if (x == p1) {
        v[1] += rho;
        v[4] += 1.0;
      }
      v[2] += 0.5 * (mx * mx + my * my + mz * mz) / rho;
      v[5] += 1.0;
    }
  }
  block_sum_store<NRED>(v, partial);
}

__global__ __launch_bounds__(BLOCK) void k_finalise(const double *__restrict__ partial, int nparts,
                                                    double *__restrict__ result, int offset) {
  double v[NRED] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nparts; b += blockDim.x)
#pragma unroll
    for (int a = 0; a < NRED; ++a) v[a] += partial[(size_t)b * NRED + a];
  __shared__ double sh[BLOCK][NRED];
#pragma unroll
  for (int a = 0; a < NRED; ++a) sh[threadIdx.x][a] = v[a];
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int a = 0; a < NRED; ++a) sh[threadIdx.x][a] += sh[threadIdx.x + s][a];
    __syncthreads();
  }
  if (threadIdx.x < NRED) result[offset + threadIdx.x] = sh[0][threadIdx.x];
}

__global__ void k_fill_zero(uint32_t *__restrict__ p, size_t n4) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Per-cell C_S field: dst == nullptr checks the FP64 input (any negative or
// non-finite entry sets *bad), otherwise converts it to the compute type.
template <typename R>
__global__ void k_set_cs(R *__restrict__ dst, const double *__restrict__ src, size_t n, int *__restrict__ bad) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double v = src[i];
    if (!dst) {
      if (!(v >= 0.0) || isinf(v)) atomicOr(bad, 1);
    } else {
      dst[i] = (R)v;
    }
  }
}

__global__ void k_header(long long *__restrict__ h, long long steps, long long q, long long N, long long storage) {
  if (threadIdx.x == 0) {
    h[0] = 0x4c424d5354415445LL;  // "LBMSTATE"
    h[1] = steps;
    h[2] = q;
    h[3] = N;
    h[4] = storage;
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
int hip_fail(lbm_ctx *ctx, hipError_t e, const char *what) {
  ctx->err = std::string(what) + ": " + hipGetErrorString(e);
  return LBM_EHIP;
}

static int check_launch(lbm_ctx *ctx, const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, what);
  return LBM_OK;
}

// Calls f.template operator()<Q, S>() for the context's lattice and storage.
template <typename F>
static int dispatch(lbm_ctx *ctx, F &&f) {
  if (ctx->q == 19) {
    if (ctx->p.storage == LBM_F64) return f.template operator()<19, double>();
    if (ctx->p.storage == LBM_F32DEV) return f.template operator()<19, float>();
    return f.template operator()<19, _Float16>();
  }
  if (ctx->p.storage == LBM_F64) return f.template operator()<27, double>();
  if (ctx->p.storage == LBM_F32DEV) return f.template operator()<27, float>();
  return f.template operator()<27, _Float16>();
}

int dev_inflow(lbm_ctx *ctx, int nvort, double sigma) {
  const int nb = (ctx->ka.ny * ctx->ka.nz + 255) / 256;
  if (ctx->p.storage == LBM_F64)
    k_inflow<double><<<nb, 256, 0, ctx->stream>>>((double *)ctx->inflow, ctx->vort, nvort, sigma, ctx->ka);
  else
    k_inflow<float><<<nb, 256, 0, ctx->stream>>>((float *)ctx->inflow, ctx->vort, nvort, sigma, ctx->ka);
  return check_launch(ctx, "k_inflow");
}

int dev_init_equilibrium(lbm_ctx *ctx, const double *rho0, const double *u0) {
  const Tiles t = tiles_of(ctx->ka);
  return dispatch(ctx, [&]<int Q, typename S>() {
    k_init_eq<Q, S><<<t.nblocks, BLOCK, 0, ctx->stream>>>((S *)ctx->pop, ctx->flags, rho0, u0, ctx->ka, t);
    return check_launch(ctx, "k_init_eq");
  });
}

template <int Q, typename S, bool ODD>
static void launch_bulk(lbm_ctx *ctx, Tiles t) {
  using R = typename Store<S>::R;
  S *pop = (S *)ctx->pop;
  const R *phi = (const R *)ctx->phi;
  // Residency cap for 4-byte storage.  K2 uses no LDS, but an LDS reservation
  // of 32 KiB per 256-thread block admits at most five blocks (five waves per
  // SIMD) on a CU's 160 KiB.  FP32 streams measurably faster at five waves
  // than at the seven to eight its register count would allow (more requests
  // in flight contend in HBM); FP16, with half the bytes per cell, is fastest
  // uncapped.
  constexpr size_t lds_cap = sizeof(S) == 4 ? 32768 : 0;
  auto go = [&](auto kern) {
    kern<<<t.nblocks, BLOCK, lds_cap, ctx->stream>>>(pop, ctx->flags, phi, ctx->ka, t, ctx->errflag);
  };
  auto by_model = [&]<bool POROUS, int SOLID>() {
    // open x faces make x non-periodic, so their domains always have solid links
    if constexpr (SOLID) {
      if (ctx->has_open) {
        if (ctx->ka.rr) go(k_bulk<Q, S, ODD, POROUS, SOLID, true, false, true>);
        else go(k_bulk<Q, S, ODD, POROUS, SOLID, false, false, true>);
        return;
      }
    }
    if (ctx->ka.rr && ctx->ka.fdw > 0.0) go(k_bulk<Q, S, ODD, POROUS, SOLID, true, true>);
    else if (ctx->ka.rr) go(k_bulk<Q, S, ODD, POROUS, SOLID, true, false>);
    else go(k_bulk<Q, S, ODD, POROUS, SOLID, false, false>);
  };
  if (ctx->porous) {
    if (ctx->has_slip) by_model.template operator()<true, 2>();
    else if (ctx->has_solid) by_model.template operator()<true, 1>();
    else by_model.template operator()<true, 0>();
  } else {
    if (ctx->has_slip) by_model.template operator()<false, 2>();
    else if (ctx->has_solid) by_model.template operator()<false, 1>();
    else by_model.template operator()<false, 0>();
  }
}

// Runs g.template operator()<ODD, SOLID>() for the current parity and
// geometry: SOLID 0 without links to leave the plain map, 1 with bounce-back
// links, 2 with full-slip faces as well.
template <typename G>
static int by_parity(lbm_ctx *ctx, G &&g) {
  const bool odd = (ctx->steps & 1) != 0;
  if (odd) {
    if (ctx->has_slip) return g.template operator()<true, 2>();
    return ctx->has_solid ? g.template operator()<true, 1>() : g.template operator()<true, 0>();
  }
  if (ctx->has_slip) return g.template operator()<false, 2>();
  return ctx->has_solid ? g.template operator()<false, 1>() : g.template operator()<false, 0>();
}

int dev_stream_probe(lbm_ctx *ctx, int n, double *ms_per_launch) {
  const Tiles t = tiles_of(ctx->ka);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(ctx, e, "hipEventCreate");
  }
  int rc = dispatch(ctx, [&]<int Q, typename S>() {
    constexpr size_t lds_cap = sizeof(S) == 4 ? 32768 : 0;  // the bulk kernel's residency cap
    auto launch = [&](bool odd) {
      S *pop = (S *)ctx->pop;
      auto go = [&](auto kern) { kern<<<t.nblocks, BLOCK, lds_cap, ctx->stream>>>(pop, ctx->flags, ctx->ka, t); };
      if (odd) {
        if (ctx->has_slip) go(k_stream_probe<Q, S, true, 2>);
        else if (ctx->has_solid) go(k_stream_probe<Q, S, true, 1>);
        else go(k_stream_probe<Q, S, true, 0>);
      } else {
        if (ctx->has_slip) go(k_stream_probe<Q, S, false, 2>);
        else if (ctx->has_solid) go(k_stream_probe<Q, S, false, 1>);
        else go(k_stream_probe<Q, S, false, 0>);
      }
    };
    launch(false);  // warm-up pair
    launch(true);
    hipError_t er = hipEventRecord(e0, ctx->stream);
    for (int i = 0; i < n && er == hipSuccess; ++i) launch((i & 1) != 0);
    if (er == hipSuccess) er = hipEventRecord(e1, ctx->stream);
    if (er == hipSuccess) er = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (er == hipSuccess) er = hipEventElapsedTime(&ms, e0, e1);
    if (er != hipSuccess) return hip_fail(ctx, er, "stream probe timing");
    *ms_per_launch = (double)ms / n;
    return check_launch(ctx, "k_stream_probe");
  });
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int dev_step(lbm_ctx *ctx) {
  const Tiles t = tiles_of(ctx->ka);
  const bool odd = (ctx->steps & 1) != 0;
  return dispatch(ctx, [&]<int Q, typename S>() {
    const int nw = ctx->nwall;
    const int wb = (nw + 255) / 256;
    const int nb = ctx->nwall_refwall;
    // hybrid collision: the step's velocity field first (read by K2 and K3 at neighbours)
    if (ctx->ka.fdw > 0.0) {
      using R = typename Store<S>::R;
      V4<R> *vel = (V4<R> *)ctx->vel;
      by_parity(ctx, [&]<bool ODD, int SOLID>() {
        k_velocity4<Q, S, ODD, SOLID><<<t.nblocks, BLOCK, 0, ctx->stream>>>((const S *)ctx->pop, ctx->flags, vel,
                                                                          ctx->ka, t);
        return LBM_OK;
      });
    }
    // wall records whose reference cell is itself a wall cell, before any wall cell is written
    if (nb > 0) {
      prof_begin(ctx, 0);
      const int lb = (nb + 255) / 256;
      auto gp = [&](auto kern) {
        kern<<<lb, 256, 0, ctx->stream>>>((const S *)ctx->pop, ctx->wmask, ctx->wcell, ctx->wref,
                                          ctx->wlist_refwall, nb, ctx->wrec, nw, ctx->ka, ctx->errflag);
      };
      if (odd) ctx->has_slip ? gp(k_wall_prepass<Q, S, true, true>) : gp(k_wall_prepass<Q, S, true, false>);
      else ctx->has_slip ? gp(k_wall_prepass<Q, S, false, true>) : gp(k_wall_prepass<Q, S, false, false>);
      prof_end(ctx, 0);
    }
    // wall cells (their reference cells are read before the bulk kernel writes them)
    if (nw > 0) {
      prof_begin(ctx, 2);
      auto gw = [&](auto kern) {
        kern<<<wb, 256, 0, ctx->stream>>>((S *)ctx->pop, ctx->wmask, ctx->wcell, ctx->wref, ctx->wrefwall, ctx->wrec,
                                          nw, ctx->ka, ctx->errflag);
      };
      if (odd) ctx->has_slip ? gw(k_wall<Q, S, true, true>) : gw(k_wall<Q, S, true, false>);
      else ctx->has_slip ? gw(k_wall<Q, S, false, true>) : gw(k_wall<Q, S, false, false>);
      prof_end(ctx, 2);
    }
    prof_begin(ctx, 1);
    if (odd) launch_bulk<Q, S, true>(ctx, t);
    else launch_bulk<Q, S, false>(ctx, t);
    prof_end(ctx, 1);
    return check_launch(ctx, "step kernels");
  });
}


int dev_velocity4(lbm_ctx *ctx) {
  const Tiles t = tiles_of(ctx->ka);
  return dispatch(ctx, [&]<int Q, typename S>() {
    using R = typename Store<S>::R;
    return by_parity(ctx, [&]<bool ODD, int SOLID>() {
      k_velocity4<Q, S, ODD, SOLID><<<t.nblocks, BLOCK, 0, ctx->stream>>>((const S *)ctx->pop, ctx->flags,
                                                                        (V4<R> *)ctx->vel, ctx->ka, t);
      return check_launch(ctx, "k_velocity4");
    });
  });
}

int dev_moments(lbm_ctx *ctx, void *rho, void *u) {
  const Tiles t = tiles_of(ctx->ka);
  return dispatch(ctx, [&]<int Q, typename S>() {
    using R = typename Store<S>::R;
    return by_parity(ctx, [&]<bool ODD, int SOLID>() {
      k_moments<Q, S, ODD, SOLID><<<t.nblocks, BLOCK, 0, ctx->stream>>>((const S *)ctx->pop, ctx->flags, (R *)rho,
                                                                        (R *)u, ctx->ka, t);
      return check_launch(ctx, "k_moments");
    });
  });
}

int dev_export(lbm_ctx *ctx, void *f) {
  const Tiles t = tiles_of(ctx->ka);
  return dispatch(ctx, [&]<int Q, typename S>() {
    using R = typename Store<S>::R;
    return by_parity(ctx, [&]<bool ODD, int SOLID>() {
      k_export<Q, S, ODD, SOLID><<<t.nblocks, BLOCK, 0, ctx->stream>>>((const S *)ctx->pop, ctx->flags, (R *)f,
                                                                       ctx->ka, t);
      return check_launch(ctx, "k_export");
    });
  });
}

int dev_import(lbm_ctx *ctx, const void *f) {
  const Tiles t = tiles_of(ctx->ka);
  return dispatch(ctx, [&]<int Q, typename S>() {
    using R = typename Store<S>::R;
    return by_parity(ctx, [&]<bool ODD, int SOLID>() {
      k_import<Q, S, ODD, SOLID><<<t.nblocks, BLOCK, 0, ctx->stream>>>((S *)ctx->pop, ctx->flags, (const R *)f,
                                                                       ctx->ka, t);
      return check_launch(ctx, "k_import");
    });
  });
}

static int reduce(lbm_ctx *ctx, int mode, int p0, int p1, int offset, double *partial, int npartial,
                  double *result) {
  const Tiles t = tiles_of(ctx->ka);
  const int grid = (int)std::min<unsigned>(t.nblocks, (unsigned)std::min(RED_BLOCKS, npartial));
  return dispatch(ctx, [&]<int Q, typename S>() {
    int rc = by_parity(ctx, [&]<bool ODD, int SOLID>() {
      k_reduce<Q, S, ODD, SOLID><<<grid, BLOCK, 0, ctx->stream>>>((const S *)ctx->pop, ctx->flags, ctx->ka, t, mode,
                                                                  p0, p1, partial);
      return check_launch(ctx, "k_reduce");
    });
    if (rc != LBM_OK) return rc;
    k_finalise<<<1, BLOCK, 0, ctx->stream>>>(partial, grid, result, offset);
    return check_launch(ctx, "k_finalise");
  });
}

int dev_reduce_diag(lbm_ctx *ctx) { return reduce(ctx, 0, -1, -1, 0, ctx->partial, ctx->npartial, ctx->result); }
int dev_objective(lbm_ctx *ctx, const int planes[2]) {
  return reduce(ctx, 1, planes[0], planes[1], 8, ctx->partial, ctx->npartial, ctx->result);
}

// ---------------------------------------------------------------------------
// Static scratch of lbm_diagnostics_noalloc: the reduction partials of at
// most RED_BLOCKS blocks and the finalised sums, in a file-scope device array
// (one copy per GPU, held until the process ends).  In host code the array's
// name is not a device address; the address comes from hipGetSymbolAddress,
// taken once per device in dev_scratch_setup and kept per device.
// ---------------------------------------------------------------------------
}  // namespace lbmk

static __device__ __align__(256) double scratch[lbmk::SCRATCH_DOUBLES];

namespace lbmk {

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

int dev_scratch_setup(lbm_ctx *ctx) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) {
    ctx->err = "device index beyond the static scratch table";
    return LBM_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(ctx, e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = ptr;
  }
  ctx->scratch = (double *)g_scratch_ptr[dev];
  return LBM_OK;
}

int dev_reduce_diag_noalloc(lbm_ctx *ctx, const double **result) {
  if (!ctx->scratch) {
    ctx->err = "static scratch not set up on this context's device";
    return LBM_EHIP;
  }
  const Tiles t = tiles_of(ctx->ka);
  const unsigned grid = std::min<unsigned>(t.nblocks, (unsigned)RED_BLOCKS);
  if ((size_t)grid * NRED + NRED > (size_t)SCRATCH_DOUBLES) {
    ctx->err = "reduction needs more partials than the static scratch holds";
    return LBM_ESIZE;
  }
  double *partial = ctx->scratch;
  double *res = ctx->scratch + (size_t)RED_BLOCKS * NRED;
  *result = res;
  return reduce(ctx, 0, -1, -1, 0, partial, RED_BLOCKS, res);
}

int dev_fill(lbm_ctx *ctx, void *ptr, size_t bytes) {
  const size_t n4 = bytes / 4;
  if (n4 == 0) return LBM_OK;
  const size_t want = (n4 + 255) / 256;
  const unsigned grid = (unsigned)std::min<size_t>(want, 65536);
  k_fill_zero<<<grid, 256, 0, ctx->stream>>>((uint32_t *)ptr, n4);
  return check_launch(ctx, "k_fill_zero");
}

int dev_set_cs(lbm_ctx *ctx, const double *cs, int *bad) {
  // the flag lives in the last slot of the workspace's result block (unused by the reductions)
  int *flag = (int *)(ctx->result + 31);
  int rc = dev_fill(ctx, flag, sizeof(int));
  if (rc != LBM_OK) return rc;
  const size_t n = (size_t)ctx->N;
  const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  // check the whole field first, so that a rejected one leaves the field in force untouched
  auto pass = [&](bool write) {
    if (ctx->p.storage == LBM_F64)
      k_set_cs<double><<<grid, 256, 0, ctx->stream>>>(write ? (double *)ctx->csf : nullptr, cs, n, flag);
    else
      k_set_cs<float><<<grid, 256, 0, ctx->stream>>>(write ? (float *)ctx->csf : nullptr, cs, n, flag);
    return check_launch(ctx, "k_set_cs");
  };
  if ((rc = pass(false)) != LBM_OK) return rc;
  hipError_t e = hipMemcpyAsync(bad, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "reading the C_S check flag");
  e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  if (*bad) return LBM_OK;
  if ((rc = pass(true)) != LBM_OK) return rc;
  e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  return LBM_OK;
}

int dev_write_header(lbm_ctx *ctx, void *dst) {
  k_header<<<1, 64, 0, ctx->stream>>>((long long *)dst, ctx->steps, ctx->q, ctx->N, ctx->p.storage);
  return check_launch(ctx, "k_header");
}

}  // namespace lbmk
