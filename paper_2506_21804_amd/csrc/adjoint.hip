// Discrete adjoint (reverse mode) of the forward step of kernels.hip, for
// gradients of a terminal objective with respect to the per-cell porosity of
// the homogenized velocity (Sec. 2.2, Eq. (12)), for both bulk collision
// models (BGK and the recursive regularized one).
//
// An adjoint field has the state's in-memory AA layout.  One reverse step
// at parity n is the transpose of the forward step: for each cell, the
// adjoints of its post-collision outputs are read from the slots the forward
// step wrote (its write set), pushed back through the collision by the
// hand-written vector-Jacobian product below, and stored into the slots the
// forward step read (its read set).  Read set = write set per cell, so the
// reverse step is in place and every cell is independent, exactly like the
// forward step; streaming and bounce-back need no code of their own.
// The Frobenius norm of the stress has no derivative at zero; its adjoint is
// taken as 0 there.
//
// Precision and storage.  Adjoint populations carry a large per-cell common
// mode (from the density terms of the objective) next to small informative
// parts.  The collision conserves mass for every state and porosity, so its
// vector-Jacobian product maps a constant vector m 1 to itself and gives it
// no porosity sensitivity: each cell takes m = mu_0 in FP64, pushes only the
// deviations mu_i - m through the product in the compute precision (FP32 for
// FP32/FP16 storage), and stores its outputs as m (one FP64 value per cell)
// plus q deviations in the compute type.  A reader recovers the value of a
// slot as the writer's m plus the stored deviation; the writer of the
// adjoint a cell reads for direction i is its downstream neighbour x + c_i,
// or the cell itself when that link is solid, at either parity.  The common
// modes are double-buffered by layout parity (readers take the previous
// step's, writers fill the current one), so no cell overwrites a value a
// neighbour still needs.  The gradient is accumulated in FP64.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "lattice.h"
#include "wall.h"

namespace lbmk {

constexpr int ATX = 64, ATY = 4, ABLOCK = ATX * ATY;

struct ATiles {
  unsigned nblocks;
  int gx, gy;
};
static ATiles atiles_of(const KArgs &k) {
  ATiles t;
  t.gx = (k.nx + ATX - 1) / ATX;
  t.gy = (k.ny + ATY - 1) / ATY;
  t.nblocks = (unsigned)t.gx * (unsigned)t.gy * (unsigned)k.nz;
  return t;
}
__device__ __forceinline__ bool atile_xyz(const KArgs &k, ATiles t, int &x, int &y, int &z) {
  const unsigned L = xcd_remap(blockIdx.x, t.nblocks);
  const int tx = (int)(L % (unsigned)t.gx);
  const unsigned r = L / (unsigned)t.gx;
  const int ty = (int)(r % (unsigned)t.gy);
  z = (int)(r / (unsigned)t.gy);
  x = tx * ATX + (int)(threadIdx.x & (ATX - 1));
  y = ty * ATY + (int)(threadIdx.x / ATX);
  return x < k.nx && y < k.ny;
}

// Vector-Jacobian product of the bulk collision in precision R.  g holds the
// state deviations, mu the adjoints of the outputs; the adjoint of input
// population i is handed to out(i, value) as soon as it is known, the
// porosity adjoint is returned and the adjoint of the cell's Smagorinsky
// coefficient smag = 18 sqrt(2) C_S^2 goes to smagb.
template <int Q, typename R, bool POROUS, typename OUT>
__device__ __forceinline__ R collide_bulk_vjp(const R g[Q], const R mu[Q], R phi, R smag, const KArgs &k, OUT out,
                                              R &smagb) {
  // ---- forward recomputation
  R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
  R mxx = R(0), myy = R(0), mzz = R(0), mxy = R(0), mxz = R(0), myz = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
    drho += g[i];
    acc(jx, cx, g[i]);
    acc(jy, cy, g[i]);
    acc(jz, cz, g[i]);
    acc(mxx, cx * cx, g[i]);
    acc(myy, cy * cy, g[i]);
    acc(mzz, cz * cz, g[i]);
    acc(mxy, cx * cy, g[i]);
    acc(mxz, cx * cz, g[i]);
    acc(myz, cy * cz, g[i]);
  }
  const R rho = R(1) + drho;
  const R ir = R(1) / rho;
  const R Fx = R(k.F[0]), Fy = R(k.F[1]), Fz = R(k.F[2]);
  const R mx = jx + R(0.5) * Fx, my = jy + R(0.5) * Fy, mz = jz + R(0.5) * Fz;
  const R ux = mx * ir, uy = my * ir, uz = mz * ir;
  const R cs2 = R(1.0 / 3.0);
  const R pxx = mxx - drho * cs2 - rho * ux * ux;
  const R pyy = myy - drho * cs2 - rho * uy * uy;
  const R pzz = mzz - drho * cs2 - rho * uz * uz;
  const R pxy = mxy - rho * ux * uy;
  const R pxz = mxz - rho * ux * uz;
  const R pyz = myz - rho * uy * uz;
  const R pn = sqrt(pxx * pxx + pyy * pyy + pzz * pzz + R(2) * (pxy * pxy + pxz * pxz + pyz * pyz));
  const R tau0 = R(k.tau0);
  const R sA = sqrt(tau0 * tau0 + smag * pn * ir);
  const R tau = R(0.5) * (tau0 + sA);
  const R om = R(1) / tau;
  const R c1 = R(1) - om, c2 = R(1) - R(0.5) * om;
  const R uu = ux * ux + uy * uy + uz * uz;
  const R vx = POROUS ? phi * ux : ux, vy = POROUS ? phi * uy : uy, vz = POROUS ? phi * uz : uz;
  const R vv = vx * vx + vy * vy + vz * vz;
  const R uF = ux * Fx + uy * Fy + uz * Fz;

  // ---- reverse through the output combination
  //   out_i = gv_i + c1 (g_i - gu_i) + c2 guo_i
  R c1b = R(0), c2b = R(0);
  R au0 = R(0), au1 = R(0), aux = R(0), auy = R(0), auz = R(0);  // equilibrium at u (and at v = u)
  R av0 = R(0), av1 = R(0), avx = R(0), avy = R(0), avz = R(0);  // equilibrium at v = phi u
  R b0 = R(0), bx = R(0), by = R(0), bz = R(0);                  // Guo term
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
    const R w = R(Lat<Q>::w(i));
    const R cu = dot3(cx, cy, cz, ux, uy, uz);
    const R cF = dot3(cx, cy, cz, Fx, Fy, Fz);
    const R eu = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
    const R gu = w * (drho + rho * eu);
    const R guo = w * (R(3) * (cF - uF) + R(9) * cu * cF);
    const R m = mu[i];
    c1b += m * (g[i] - gu);
    c2b += m * guo;
    // adjoint weights of gu (-c1 m), gv (m) and guo (c2 m), each times w
    const R su = POROUS ? -c1 * m * w : (R(1) - c1) * m * w;
    au0 += su;
    au1 += su * eu;
    const R tu = su * (R(3) + R(9) * cu);
    acc(aux, cx, tu);
    acc(auy, cy, tu);
    acc(auz, cz, tu);
    if (POROUS) {
      const R sv = m * w;
      const R cv = dot3(cx, cy, cz, vx, vy, vz);
      av0 += sv;
      av1 += sv * (R(3) * cv + R(4.5) * cv * cv - R(1.5) * vv);
      const R tv = sv * (R(3) + R(9) * cv);
      acc(avx, cx, tv);
      acc(avy, cy, tv);
      acc(avz, cz, tv);
    }
    const R sg = c2 * m * w;
    b0 += sg;
    const R tg = sg * R(9) * cF;
    acc(bx, cx, tg);
    acc(by, cy, tg);
    acc(bz, cz, tg);
  }
  // equilibria: d/d drho = w, d/d rho = w (3cv + 9/2 cv^2 - 3/2 v.v), d/dv = w rho (3c + 9 (c.v) c - 3 v)
  R drhob = au0;
  R rhob = au1;
  R uxb = rho * aux - R(3) * rho * ux * au0;
  R uyb = rho * auy - R(3) * rho * uy * au0;
  R uzb = rho * auz - R(3) * rho * uz * au0;
  R phib = R(0);
  if (POROUS) {
    drhob += av0;
    rhob += av1;
    const R vxb = rho * avx - R(3) * rho * vx * av0;
    const R vyb = rho * avy - R(3) * rho * vy * av0;
    const R vzb = rho * avz - R(3) * rho * vz * av0;
    uxb += phi * vxb;
    uyb += phi * vyb;
    uzb += phi * vzb;
    phib = vxb * ux + vyb * uy + vzb * uz;
  }
  // Guo term: d/du = w (-3 F + 9 (c.F) c)
  uxb += bx - R(3) * Fx * b0;
  uyb += by - R(3) * Fy * b0;
  uzb += bz - R(3) * Fz * b0;
  // relaxation rate: om = 1/tau, tau = (tau0 + sqrt(A))/2, A = tau0^2 + smag pn / rho
  const R omb = -c1b - R(0.5) * c2b;
  const R taub = -omb * om * om;
  const R Ab = R(0.5) * taub / (R(2) * sA);
  const R pnb = Ab * smag * ir;
  R irb = Ab * smag * pn;
  smagb = Ab * pn * ir;
  const R q = pn > R(0) ? pnb / pn : R(0);  // d pn / d P_ab = P_ab / pn (off-diagonals twice)
  const R pxxb = q * pxx, pyyb = q * pyy, pzzb = q * pzz;
  const R pxyb = R(2) * q * pxy, pxzb = R(2) * q * pxz, pyzb = R(2) * q * pyz;
  drhob -= cs2 * (pxxb + pyyb + pzzb);
  rhob -= ux * ux * pxxb + uy * uy * pyyb + uz * uz * pzzb + ux * uy * pxyb + ux * uz * pxzb + uy * uz * pyzb;
  uxb -= rho * (R(2) * ux * pxxb + uy * pxyb + uz * pxzb);
  uyb -= rho * (R(2) * uy * pyyb + ux * pxyb + uz * pyzb);
  uzb -= rho * (R(2) * uz * pzzb + ux * pxzb + uy * pyzb);
  // u = m / rho
  const R mxb = uxb * ir, myb = uyb * ir, mzb = uzb * ir;
  irb += uxb * mx + uyb * my + uzb * mz;
  rhob -= irb * ir * ir;
  drhob += rhob;
  // moments -> populations, plus the direct c1 path of g_i
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
    R s = drhob + c1 * mu[i];
    acc(s, cx, mxb);
    acc(s, cy, myb);
    acc(s, cz, mzb);
    acc(s, cx * cx, pxxb);
    acc(s, cy * cy, pyyb);
    acc(s, cz * cz, pzzb);
    acc(s, cx * cy, pxyb);
    acc(s, cx * cz, pxzb);
    acc(s, cy * cz, pyzb);
    out(i, s);
  }
  return phib;
}

// Vector-Jacobian product of the recursive regularized collision (the
// RR = true branch of collide_bulk) in precision R.  Forward:
//   out_i = w_i (drho + rho (3 c.v + 9/2 (c.v)^2 - 3/2 v.v)) + w_i T3(rho v v v)_i
//         + c1 [ -3/2 w_i c.F + 9/2 w_i (c.Pi.c - c_s^2 tr Pi) + w_i T3(A1(u, Pi))_i ]
//         + c2 w_i (3 (c.F - u.F) + 9 (c.u)(c.F)),
// with u = (j + F/2)/rho, Pi = M2 - drho c_s^2 I - rho u u, v = phi u,
// c1 = 1 - 1/tau, c2 = 1 - 1/(2 tau), tau from |Pi| and rho, and T3 the
// projection on the lattice's third-order Hermite basis (linear in its
// tensor argument: sum_i mu_i w_i T3(A)_i = sum_k <A, P_k> M_k / |P_k|^2 with
// M_k = sum_i mu_i w_i P_k(c_i)).  The outputs depend on g only through its
// moments.
//
// HYB = true: the hybrid of Eq. (7) with the finite-difference strain Sfd of
// the step's velocity field: the second-order coefficient is
// h = sigma Pi - fs Sfd, fs = (1 - sigma) 2 rho c_s^2 tau, and the third-order
// part keeps the factor sigma; the adjoint of Sfd (its six components) goes
// to Sb.
template <int Q, typename R, bool POROUS, bool HYB = false, typename OUT>
__device__ __forceinline__ R collide_bulk_rr_vjp(const R g[Q], const R mu[Q], R phi, R smag, const KArgs &k, OUT out,
                                                 R &smagb, const R *Sfd = nullptr, R *Sb = nullptr) {
  // ---- forward recomputation
  R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
  R mxx = R(0), myy = R(0), mzz = R(0), mxy = R(0), mxz = R(0), myz = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
    drho += g[i];
    acc(jx, cx, g[i]);
    acc(jy, cy, g[i]);
    acc(jz, cz, g[i]);
    acc(mxx, cx * cx, g[i]);
    acc(myy, cy * cy, g[i]);
    acc(mzz, cz * cz, g[i]);
    acc(mxy, cx * cy, g[i]);
    acc(mxz, cx * cz, g[i]);
    acc(myz, cy * cz, g[i]);
  }
  const R rho = R(1) + drho;
  const R ir = R(1) / rho;
  const R Fx = R(k.F[0]), Fy = R(k.F[1]), Fz = R(k.F[2]);
  const R mx = jx + R(0.5) * Fx, my = jy + R(0.5) * Fy, mz = jz + R(0.5) * Fz;
  const R ux = mx * ir, uy = my * ir, uz = mz * ir;
  const R cs2 = R(1.0 / 3.0);
  const R pxx = mxx - drho * cs2 - rho * ux * ux;
  const R pyy = myy - drho * cs2 - rho * uy * uy;
  const R pzz = mzz - drho * cs2 - rho * uz * uz;
  const R pxy = mxy - rho * ux * uy;
  const R pxz = mxz - rho * ux * uz;
  const R pyz = myz - rho * uy * uz;
  const R pn = sqrt(pxx * pxx + pyy * pyy + pzz * pzz + R(2) * (pxy * pxy + pxz * pxz + pyz * pyz));
  const R tau0 = R(k.tau0);
  const R sA = sqrt(tau0 * tau0 + smag * pn * ir);
  const R tau = R(0.5) * (tau0 + sA);
  const R om = R(1) / tau;
  const R c1 = R(1) - om, c2 = R(1) - R(0.5) * om;
  const R vx = POROUS ? phi * ux : ux, vy = POROUS ? phi * uy : uy, vz = POROUS ? phi * uz : uz;
  const R vv = vx * vx + vy * vy + vz * vz;
  const R uF = ux * Fx + uy * Fy + uz * Fz;
  R sig = R(1), fs = R(0);
  R hxx = pxx, hyy = pyy, hzz = pzz, hxy = pxy, hxz = pxz, hyz = pyz;  // second-order coefficient
  if constexpr (HYB) {
    const R fw = R(k.fdw);
    sig = R(1) - fw;
    fs = fw * R(2.0 / 3.0) * rho * tau;
    hxx = sig * pxx - fs * Sfd[0];
    hyy = sig * pyy - fs * Sfd[1];
    hzz = sig * pzz - fs * Sfd[2];
    hxy = sig * pxy - fs * Sfd[3];
    hxz = sig * pxz - fs * Sfd[4];
    hyz = sig * pyz - fs * Sfd[5];
  }
  const R tr3 = (hxx + hyy + hzz) * cs2;
  R A1[7], K1[7];
  A1[0] = R(2) * ux * pxy + uy * pxx;
  A1[1] = R(2) * ux * pxz + uz * pxx;
  A1[2] = R(2) * uy * pxy + ux * pyy;
  A1[3] = R(2) * uy * pyz + uz * pyy;
  A1[4] = R(2) * uz * pxz + ux * pzz;
  A1[5] = R(2) * uz * pyz + uy * pzz;
  A1[6] = ux * pyz + uy * pxz + uz * pxy;
  third_coefs<Q, R>(A1, K1);

  // ---- reverse through the outputs
  R c1b = R(0), c2b = R(0);
  R s0 = R(0), s1 = R(0);                      // sum mu w, sum mu w (3cv + 9/2 cv^2 - 3/2 vv)
  R evx = R(0), evy = R(0), evz = R(0);        // sum mu w (3 + 9 c.v) c
  R gux = R(0), guy = R(0), guz = R(0);        // sum mu w (9 c.F) c   (Guo, times c2 later)
  R gF = R(0);                                 // sum mu w
  R pbxx = R(0), pbyy = R(0), pbzz = R(0), pbxy = R(0), pbxz = R(0), pbyz = R(0), pbtr = R(0);
  R M[7];
#pragma unroll
  for (int m = 0; m < 7; ++m) M[m] = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
    const R w = R(Lat<Q>::w(i));
    const R mw = mu[i] * w;
    const R cu = dot3(cx, cy, cz, ux, uy, uz);
    const R cv = dot3(cx, cy, cz, vx, vy, vz);
    const R cF = dot3(cx, cy, cz, Fx, Fy, Fz);
    R cPc = R(0);
    acc(cPc, cx * cx, hxx);
    acc(cPc, cy * cy, hyy);
    acc(cPc, cz * cz, hzz);
    acc(cPc, cx * cy, R(2) * hxy);
    acc(cPc, cx * cz, R(2) * hxz);
    acc(cPc, cy * cz, R(2) * hyz);
    const R t1 = third_term<Q, R>(i, K1);
    c1b += mw * (R(-1.5) * cF + R(4.5) * (cPc - tr3) + sig * t1);
    c2b += mw * (R(3) * (cF - uF) + R(9) * cu * cF);
    s0 += mw;
    s1 += mw * (R(3) * cv + R(4.5) * cv * cv - R(1.5) * vv);
    const R te = mw * (R(3) + R(9) * cv);
    acc(evx, cx, te);
    acc(evy, cy, te);
    acc(evz, cz, te);
    const R tg = mw * R(9) * cF;
    acc(gux, cx, tg);
    acc(guy, cy, tg);
    acc(guz, cz, tg);
    gF += mw;
    // 9/2 w (c.Pi.c - c_s^2 tr Pi): d/dp_aa = 9/2 w c_a^2, d/dp_ab = 9 w c_a c_b, tr part separately
    acc(pbxx, cx * cx, mw);
    acc(pbyy, cy * cy, mw);
    acc(pbzz, cz * cz, mw);
    acc(pbxy, cx * cy, mw);
    acc(pbxz, cx * cz, mw);
    acc(pbyz, cy * cz, mw);
    pbtr += mw;
#pragma unroll
    for (int kk = 0; kk < H3Basis<Q>::n; ++kk) {
      const double pk = H3Basis<Q>::P(kk, i);
      if (pk != 0.0) M[kk] += mw * R(pk);
    }
  }
  // adjoints of the tensor components through the projection: Ab = sum_k M_k / |P_k|^2 d<A,P_k>/dA
  R Ab[7];
  {
    constexpr H3Norms<Q> nrm = h3_norms<Q>();
#pragma unroll
    for (int m = 0; m < 7; ++m) Ab[m] = R(0);
#pragma unroll
    for (int kk = 0; kk < H3Basis<Q>::n; ++kk) {
      const R mk = M[kk] * R(1.0 / nrm.v[kk]);
      Ab[H3Basis<Q>::c0(kk)] += mk;
      if (H3Basis<Q>::sgn(kk) > 0.0) Ab[H3Basis<Q>::c1(kk)] += mk;
      if (H3Basis<Q>::sgn(kk) < 0.0) Ab[H3Basis<Q>::c1(kk)] -= mk;
    }
  }
  // equilibrium: drho, rho and v
  R drhob = s0;
  R rhob = s1;
  R vxb = rho * (evx - R(3) * vx * s0), vyb = rho * (evy - R(3) * vy * s0), vzb = rho * (evz - R(3) * vz * s0);
  // third-order equilibrium A0 = rho v v v:
  // xxy, xxz, xyy, yyz, xzz, yzz, xyz
  rhob += Ab[0] * vx * vx * vy + Ab[1] * vx * vx * vz + Ab[2] * vx * vy * vy + Ab[3] * vy * vy * vz +
          Ab[4] * vx * vz * vz + Ab[5] * vy * vz * vz + Ab[6] * vx * vy * vz;
  vxb += rho * (Ab[0] * R(2) * vx * vy + Ab[1] * R(2) * vx * vz + Ab[2] * vy * vy + Ab[4] * vz * vz + Ab[6] * vy * vz);
  vyb += rho * (Ab[0] * vx * vx + Ab[2] * R(2) * vx * vy + Ab[3] * R(2) * vy * vz + Ab[5] * vz * vz + Ab[6] * vx * vz);
  vzb += rho * (Ab[1] * vx * vx + Ab[3] * vy * vy + Ab[4] * R(2) * vx * vz + Ab[5] * R(2) * vy * vz + Ab[6] * vx * vy);
  // regularized f^(1), times c1: the second-order coefficient directly, and Pi and u through A1
  R pxxb = c1 * R(4.5) * (pbxx - cs2 * pbtr), pyyb = c1 * R(4.5) * (pbyy - cs2 * pbtr),
    pzzb = c1 * R(4.5) * (pbzz - cs2 * pbtr);
  R pxyb = c1 * R(9) * pbxy, pxzb = c1 * R(9) * pbxz, pyzb = c1 * R(9) * pbyz;
  R tau_h = R(0);  // adjoint of tau through fs (hybrid)
  if constexpr (HYB) {
    // h = sigma Pi - fs Sfd: to Sfd, to fs (then rho and tau), and sigma to Pi
    const R fsb = -(pxxb * Sfd[0] + pyyb * Sfd[1] + pzzb * Sfd[2] + pxyb * Sfd[3] + pxzb * Sfd[4] + pyzb * Sfd[5]);
    Sb[0] = -fs * pxxb;
    Sb[1] = -fs * pyyb;
    Sb[2] = -fs * pzzb;
    Sb[3] = -fs * pxyb;
    Sb[4] = -fs * pxzb;
    Sb[5] = -fs * pyzb;
    pxxb *= sig;
    pyyb *= sig;
    pzzb *= sig;
    pxyb *= sig;
    pxzb *= sig;
    pyzb *= sig;
    const R fw = R(k.fdw);
    rhob += fsb * fw * R(2.0 / 3.0) * tau;
    tau_h = fsb * fw * R(2.0 / 3.0) * rho;
  }
  R uxb = R(0), uyb = R(0), uzb = R(0);
  {
    R B[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) B[m] = c1 * sig * Ab[m];
    // A1: xxy = 2 ux pxy + uy pxx; xxz = 2 ux pxz + uz pxx; xyy = 2 uy pxy + ux pyy;
    //     yyz = 2 uy pyz + uz pyy; xzz = 2 uz pxz + ux pzz; yzz = 2 uz pyz + uy pzz;
    //     xyz = ux pyz + uy pxz + uz pxy
    uxb += B[0] * R(2) * pxy + B[1] * R(2) * pxz + B[2] * pyy + B[4] * pzz + B[6] * pyz;
    uyb += B[0] * pxx + B[2] * R(2) * pxy + B[3] * R(2) * pyz + B[5] * pzz + B[6] * pxz;
    uzb += B[1] * pxx + B[3] * pyy + B[4] * R(2) * pxz + B[5] * R(2) * pyz + B[6] * pxy;
    pxxb += B[0] * uy + B[1] * uz;
    pyyb += B[2] * ux + B[3] * uz;
    pzzb += B[4] * ux + B[5] * uy;
    pxyb += B[0] * R(2) * ux + B[2] * R(2) * uy + B[6] * uz;
    pxzb += B[1] * R(2) * ux + B[4] * R(2) * uz + B[6] * uy;
    pyzb += B[3] * R(2) * uy + B[5] * R(2) * uz + B[6] * ux;
  }
  // Guo term, times c2: d/du = w (-3 F + 9 (c.F) c)
  uxb += c2 * (gux - R(3) * Fx * gF);
  uyb += c2 * (guy - R(3) * Fy * gF);
  uzb += c2 * (guz - R(3) * Fz * gF);
  // homogenized velocity
  R phib = R(0);
  if (POROUS) {
    uxb += phi * vxb;
    uyb += phi * vyb;
    uzb += phi * vzb;
    phib = vxb * ux + vyb * uy + vzb * uz;
  } else {
    uxb += vxb;
    uyb += vyb;
    uzb += vzb;
  }
  // relaxation rate: om = 1/tau, tau = (tau0 + sqrt(A))/2, A = tau0^2 + smag pn / rho
  const R omb = -c1b - R(0.5) * c2b;
  const R taub = -omb * om * om + tau_h;
  const R Abar = R(0.5) * taub / (R(2) * sA);
  const R pnb = Abar * smag * ir;
  R irb = Abar * smag * pn;
  smagb = Abar * pn * ir;
  const R q = pn > R(0) ? pnb / pn : R(0);
  pxxb += q * pxx;
  pyyb += q * pyy;
  pzzb += q * pzz;
  pxyb += R(2) * q * pxy;
  pxzb += R(2) * q * pxz;
  pyzb += R(2) * q * pyz;
  // Pi = M2 - drho c_s^2 I - rho u u
  drhob -= cs2 * (pxxb + pyyb + pzzb);
  rhob -= ux * ux * pxxb + uy * uy * pyyb + uz * uz * pzzb + ux * uy * pxyb + ux * uz * pxzb + uy * uz * pyzb;
  uxb -= rho * (R(2) * ux * pxxb + uy * pxyb + uz * pxzb);
  uyb -= rho * (R(2) * uy * pyyb + ux * pxyb + uz * pyzb);
  uzb -= rho * (R(2) * uz * pzzb + ux * pxzb + uy * pyzb);
  // u = m / rho
  const R mxb = uxb * ir, myb = uyb * ir, mzb = uzb * ir;
  irb += uxb * mx + uyb * my + uzb * mz;
  rhob -= irb * ir * ir;
  drhob += rhob;
  // moments -> populations
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
    R s = drhob;
    acc(s, cx, mxb);
    acc(s, cy, myb);
    acc(s, cz, mzb);
    acc(s, cx * cx, pxxb);
    acc(s, cy * cy, pyyb);
    acc(s, cz * cz, pzzb);
    acc(s, cx * cy, pxyb);
    acc(s, cx * cz, pxzb);
    acc(s, cy * cz, pyzb);
    out(i, s);
  }
  return phib;
}

// Cell that wrote the adjoint that cell n reads for direction i (see above).
template <int Q, int SOLID>
__device__ __forceinline__ int writer_of(const Nb &n, LinkMask sm, int i) {
  if (SOLID && ((sm >> Lat<Q>::opp(i)) & 1u)) return n.cell;
  // across full-slip faces: the cell the reflected population arrives at
  if (SOLID == 2 && ((sm >> (32 + Lat<Q>::opp(i))) & 1u))
    return n.cell + reflect_off<Q>(n, i, +1, face_axes(cross_faces<Q>(n, i, +1)));
  return n.cell + nb_off<Q>(n, i, +1);
}

// Open x faces: the rebuild of an inlet or outlet cell's pre-collision
// deviations (the same map as in the bulk kernel: regularized inlet at the
// prescribed velocity, equilibrium outlet at rho_out) and the transpose of
// its Jacobian.  With n the outward normal, the known populations are those
// with c.n >= 0; m = G_0 + 2 G_+ sums them (G_0 over c.n = 0, G_+ over the
// ones leaving through the face), and rho (1 + u.n) = 1 + m.
template <int Q, typename R, bool RR>
struct OpenMap {
  static constexpr int H = (Q - 1) / 2;
  bool outlet;
  int nxo;                  // x component of the outward normal
  R drho, rho, ux, uy, uz;  // rebuilt density and velocity
  R K[7];                   // third-order coefficients of the unit-density equilibrium (RR)
  __device__ __forceinline__ OpenMap(const R g[Q], bool out, int y, int z, const KArgs &k) : outlet(out) {
    nxo = outlet ? 1 : -1;
    R m = g[0];
#pragma unroll
    for (int i = 1; i <= H; ++i) {
      const int cx = Lat<Q>::c(i, 0);
      if (cx == 0) m += g[i] + g[i + H];
      else m += R(2) * (cx * nxo > 0 ? g[i] : g[i + H]);
    }
    uy = R(0);
    uz = R(0);
    if (outlet) {
      drho = R(k.rho_out - 1.0);
      rho = R(1) + drho;
      ux = (m - drho) / rho;
    } else {
      const R *f = static_cast<const R *>(k.inflow);
      const int face = k.ny * k.nz, c2 = y + k.ny * z;
      ux = f[c2];
      uy = f[face + c2];
      uz = f[2 * face + c2];
      drho = (m + ux) / (R(1) - ux);  // u.n = -ux
      rho = R(1) + drho;
    }
    if constexpr (RR) {
      R A[7];
      cube_tensor(R(1), ux, uy, uz, A);
      third_coefs<Q, R>(A, K);
    }
  }
  // unit-density equilibrium parts of direction i <= H: even e, odd o
  // (f^eq_i - w_i = w_i (drho + rho (e + o)), f^eq_ibar: o -> -o)
  __device__ __forceinline__ void unit(int i, R &e, R &o) const {
    const R cu = dot3(Lat<Q>::c(i, 0), Lat<Q>::c(i, 1), Lat<Q>::c(i, 2), ux, uy, uz);
    const R uu = ux * ux + uy * uy + uz * uz;
    e = R(4.5) * cu * cu - R(1.5) * uu;
    o = R(3) * cu;
    if constexpr (RR) o += third_term<Q, R>(i, K);
  }
  __device__ __forceinline__ void geq(R out[Q]) const {
    const R uu = ux * ux + uy * uy + uz * uz;
    out[0] = R(Lat<Q>::w(0)) * (drho - R(1.5) * rho * uu);
#pragma unroll
    for (int i = 1; i <= H; ++i) {
      R e, o;
      unit(i, e, o);
      const R w = R(Lat<Q>::w(i));
      out[i] = w * (drho + rho * (e + o));
      out[i + H] = w * (drho + rho * (e - o));
    }
  }
  // rebuilt deviations
  __device__ __forceinline__ void forward(const R g[Q], R out[Q]) const {
    geq(out);
    if (outlet) return;
    R pxx = R(0), pyy = R(0), pzz = R(0), pxy = R(0), pxz = R(0), pyz = R(0);
#pragma unroll
    for (int i = 1; i <= H; ++i) {
      const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
      R hs;
      if (cx == 0) {
        hs = (g[i] - out[i]) + (g[i + H] - out[i + H]);
      } else {
        const int kn = cx * nxo > 0 ? i : i + H;
        hs = R(2) * (g[kn] - out[kn]);
      }
      acc(pxx, cx * cx, hs);
      acc(pyy, cy * cy, hs);
      acc(pzz, cz * cz, hs);
      acc(pxy, cx * cy, hs);
      acc(pxz, cx * cz, hs);
      acc(pyz, cy * cz, hs);
    }
    const R tr3 = (pxx + pyy + pzz) * R(1.0 / 3.0);
    out[0] -= R(4.5) * R(Lat<Q>::w(0)) * tr3;
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
      out[i] += r;
      out[i + H] += r;
    }
  }
  // b: adjoint of the rebuilt deviations in, adjoint of the gathered ones out
  // (the map is affine in the known populations at the inlet; at the outlet
  // only through u.n, where this is the Jacobian at the current state)
  __device__ __forceinline__ void transpose(R b[Q]) const {
    R gb[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) gb[i] = R(0);
    R mb;
    if (outlet) {
      // f^eq_i(rho_out, (ux, 0, 0)): d/dux = w_i rho (3 c_x + 9 c_x^2 ux - 3 ux)
      R uxb = R(0);
#pragma unroll
      for (int i = 1; i <= H; ++i) {
        const R cx = R(Lat<Q>::c(i, 0));
        const R w = R(Lat<Q>::w(i));
        const R ev = R(9) * cx * cx * ux - R(3) * ux, od = R(3) * cx;
        uxb += w * rho * ((ev + od) * b[i] + (ev - od) * b[i + H]);
      }
      uxb += R(Lat<Q>::w(0)) * rho * (-R(3) * ux) * b[0];
      mb = uxb / rho;
    } else {
      // Pi adjoint: out_i += 9/2 w_i (c.Pi.c - tr Pi / 3)
      R bxx = R(0), byy = R(0), bzz = R(0), bxy = R(0), bxz = R(0), byz = R(0);
      const R third = R(1.0 / 3.0);
      {
        const R t = R(4.5) * R(Lat<Q>::w(0)) * b[0];
        bxx -= t * third;
        byy -= t * third;
        bzz -= t * third;
      }
#pragma unroll
      for (int i = 1; i <= H; ++i) {
        const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
        const R t = R(4.5) * R(Lat<Q>::w(i)) * (b[i] + b[i + H]);
        bxx += t * (R(cx * cx) - third);
        byy += t * (R(cy * cy) - third);
        bzz += t * (R(cz * cz) - third);
        bxy += t * R(2 * cx * cy);
        bxz += t * R(2 * cx * cz);
        byz += t * R(2 * cy * cz);
      }
      // geq adjoint starts as b; the pair sums take the Pi adjoint back
      R geqb[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) geqb[i] = b[i];
#pragma unroll
      for (int i = 1; i <= H; ++i) {
        const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
        R hsb = R(0);
        acc(hsb, cx * cx, bxx);
        acc(hsb, cy * cy, byy);
        acc(hsb, cz * cz, bzz);
        acc(hsb, cx * cy, bxy);
        acc(hsb, cx * cz, bxz);
        acc(hsb, cy * cz, byz);
        if (cx == 0) {
          gb[i] += hsb;
          gb[i + H] += hsb;
          geqb[i] -= hsb;
          geqb[i + H] -= hsb;
        } else {
          const int kn = cx * nxo > 0 ? i : i + H;
          gb[kn] += R(2) * hsb;
          geqb[kn] -= R(2) * hsb;
        }
      }
      // f^eq at the prescribed velocity depends on drho only:
      // d f^eq_i / d drho = w_i (1 + e + o)
      R drhob = R(Lat<Q>::w(0)) * (R(1) - R(1.5) * (ux * ux + uy * uy + uz * uz)) * geqb[0];
#pragma unroll
      for (int i = 1; i <= H; ++i) {
        R e, o;
        unit(i, e, o);
        const R w = R(Lat<Q>::w(i));
        drhob += w * ((R(1) + e + o) * geqb[i] + (R(1) + e - o) * geqb[i + H]);
      }
      mb = drhob / (R(1) - ux);
    }
    // m = G_0 + 2 G_+
    gb[0] += mb;
#pragma unroll
    for (int i = 1; i <= H; ++i) {
      const int cx = Lat<Q>::c(i, 0);
      if (cx == 0) {
        gb[i] += mb;
        gb[i + H] += mb;
      } else {
        gb[cx * nxo > 0 ? i : i + H] += R(2) * mb;
      }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) b[i] = gb[i];
  }
};

// Seed of the objective J = c_s^2 (<rho>_{x=p0} - <rho>_{x=p1}) + <rho |u|^2 / 2>
// at one cell, scaled by w: the part common to all populations (the density
// terms) and the kinetic-energy part of population i, (c_i.u - |u|^2/2) / n_fluid.
struct CellSeed {
  double base, ux, uy, uz, uu, inf;
  template <int Q>
  __device__ __forceinline__ double kin(int i) const {
    return (dot3(Lat<Q>::c(i, 0), Lat<Q>::c(i, 1), Lat<Q>::c(i, 2), ux, uy, uz) - 0.5 * uu) * inf;
  }
};
template <int Q, typename R>
__device__ __forceinline__ CellSeed cell_seed(const R g[Q], int x, int p0, int p1, const double *cnt, double w,
                                              const KArgs &k) {
  double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double gi = (double)g[i];
    drho += gi;
    acc(jx, Lat<Q>::c(i, 0), gi);
    acc(jy, Lat<Q>::c(i, 1), gi);
    acc(jz, Lat<Q>::c(i, 2), gi);
  }
  const double rho = 1.0 + drho;
  CellSeed c;
  c.ux = (jx + 0.5 * k.F[0]) / rho;
  c.uy = (jy + 0.5 * k.F[1]) / rho;
  c.uz = (jz + 0.5 * k.F[2]) / rho;
  c.uu = c.ux * c.ux + c.uy * c.uy + c.uz * c.uz;
  c.base = 0.0;
  if (x == p0) c.base += w / (3.0 * cnt[0]);
  if (x == p1) c.base -= w / (3.0 * cnt[1]);
  c.inf = w / cnt[2];
  return c;
}

// SEED = true (time-averaged objectives): the step also adds w dJ/df of the
// state it reads (the objective's seed at that step), after the transpose.
// HYB = true (hybrid collision, with RR): the finite-difference strain of the
// step's velocity field (k.vel) is held fixed here and its adjoint written to
// sbar[6][N]; k_adjoint_fd then carries it to the velocities it came from.
template <int Q, typename S, bool ODD, bool POROUS, int SOLID, bool RR, bool SEED = false, bool OPEN = false,
          bool HYB = false>
__global__ __launch_bounds__(ABLOCK) void k_adjoint(const S *__restrict__ pop, const uint8_t *__restrict__ flags,
                                                    typename Store<S>::R *__restrict__ dev,
                                                    const double *__restrict__ m_prev, double *__restrict__ m_next,
                                                    const typename Store<S>::R *__restrict__ phi,
                                                    double *__restrict__ grad, double *__restrict__ gcs, KArgs k,
                                                    ATiles t, int p0 = 0, int p1 = 0,
                                                    const double *__restrict__ cnt = nullptr, double sw = 0.0,
                                                    typename Store<S>::R *__restrict__ sbar = nullptr) {
  using R = typename Store<S>::R;
  static_assert(!HYB || (RR && !OPEN), "the hybrid collision comes with RR and without open faces");
  int x, y, z;
  if (!atile_xyz(k, t, x, y, z)) return;
  const Nb n = make_nb(x, y, z, k);
  const uint8_t fl = flags[n.cell];
  // wall cells have a reverse kernel of their own (k_adjoint_wall)
  if (!(fl & FL_FLUID) || (fl & FL_WALL)) return;
  LinkMask sm = 0;
  if (SOLID && (fl & FL_NEAR)) sm = solid_mask<Q, SOLID == 2>(n, flags);
  const size_t N = (size_t)k.N;
  if (fl & FL_LID) {
    // the lid output does not depend on the state: only the seed remains
    if constexpr (SEED) {
      R g[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) g[i] = Store<S>::ld(pop + read_slot<Q, ODD, SOLID == 2>(n, sm, i, N));
      const CellSeed cs = cell_seed<Q, R>(g, x, p0, p1, cnt, sw, k);
#pragma unroll
      for (int i = 0; i < Q; ++i) dev[read_slot<Q, ODD, SOLID == 2>(n, sm, i, N)] = (R)cs.template kin<Q>(i);
      m_next[n.cell] = cs.base;
      return;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) dev[read_slot<Q, ODD, SOLID == 2>(n, sm, i, N)] = R(0);
    m_next[n.cell] = 0.0;
    return;
  }
  double scale = 1.0;
  // the outlet plane is left out of the fringe
  if (x >= k.fringe_start && !(OPEN && (fl & FL_OUTLET))) scale = 1.0 - (double)static_cast<const R *>(k.lam)[x];
  // mu_i = scale (M[writer_i] + d_i); the rest direction's writer is the cell itself
  const double mx = m_prev[n.cell];
  const double d0 = (double)dev[write_slot<Q, ODD, SOLID == 2>(n, sm, 0, N)];
  const double m = scale * (mx + d0);
  R dmu[Q];
  dmu[0] = R(0);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const double mw = m_prev[writer_of<Q, SOLID>(n, sm, i)];
    const double di = (double)dev[write_slot<Q, ODD, SOLID == 2>(n, sm, i, N)];
    dmu[i] = (R)(scale * ((mw - mx) + (di - d0)));
  }
  R g[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) g[i] = Store<S>::ld(pop + read_slot<Q, ODD, SOLID == 2>(n, sm, i, N));
  const R ph = POROUS ? phi[n.cell] : R(1);
  CellSeed cs{};
  if constexpr (SEED) cs = cell_seed<Q, R>(g, x, p0, p1, cnt, sw, k);
  auto store = [&](int i, R v) {
    if constexpr (SEED) v += (R)cs.template kin<Q>(i);
    dev[read_slot<Q, ODD, SOLID == 2>(n, sm, i, N)] = v;
  };
  const R smag = smag_of<R>(k, n.cell);
  R phib, smagb;
  // dJ/dC_S of the cell (gcs != NULL): smag = 18 sqrt(2) C_S^2
  auto add_cs = [&]() {
    if (gcs) gcs[n.cell] += (double)smagb * (2.0 * SMAG_COEF) * cs_of<R>(k, n.cell);
  };
  if constexpr (OPEN) {
    if (fl & (FL_INLET | FL_OUTLET)) {
      // open face: the collision acts on the rebuilt populations; the
      // adjoint of the gathered ones is the transpose of the rebuild applied
      // to m 1 + (VJP deviations), its common part taken in FP64
      const OpenMap<Q, R, RR> om(g, (fl & FL_OUTLET) != 0, y, z, k);
      R gre[Q];
      om.forward(g, gre);
      R ob[Q], one[Q];
      auto collect = [&](int i, R v) { ob[i] = v; };
      if constexpr (RR) phib = collide_bulk_rr_vjp<Q, R, POROUS>(gre, dmu, ph, smag, k, collect, smagb);
      else phib = collide_bulk_vjp<Q, R, POROUS>(gre, dmu, ph, smag, k, collect, smagb);
#pragma unroll
      for (int i = 0; i < Q; ++i) one[i] = R(1);
      om.transpose(ob);
      om.transpose(one);
#pragma unroll
      for (int i = 0; i < Q; ++i) store(i, (R)(m * ((double)one[i] - 1.0)) + ob[i]);
      m_next[n.cell] = SEED ? m + cs.base : m;
      if (POROUS) grad[n.cell] += (double)phib;
      add_cs();
      return;
    }
  }
  if constexpr (HYB) {
    R Sfd[6], Sb[6];
    fd_strain<R>(n, k, Sfd);
    phib = collide_bulk_rr_vjp<Q, R, POROUS, true>(g, dmu, ph, smag, k, store, smagb, Sfd, Sb);
#pragma unroll
    for (int m = 0; m < 6; ++m) sbar[(size_t)m * N + n.cell] = Sb[m];
  } else if constexpr (RR) {
    phib = collide_bulk_rr_vjp<Q, R, POROUS>(g, dmu, ph, smag, k, store, smagb);
  } else {
    phib = collide_bulk_vjp<Q, R, POROUS>(g, dmu, ph, smag, k, store, smagb);
  }
  m_next[n.cell] = SEED ? m + cs.base : m;
  if (POROUS) grad[n.cell] += (double)phib;
  add_cs();
}

// ---------------------------------------------------------------------------
// Wall model (Sec. 2.2.1).  A wall cell's output depends on its own
// populations and, through its record (t, u_tan, G, tau_b), on the velocity
// of its reference cell.  The reverse step of a wall cell pushes the adjoint
// of its outputs back through the reconstruction collision to its own
// populations, and through the record to the reference cell's density and
// momentum; a second pass adds the latter to the reference cells' adjoints.
// ---------------------------------------------------------------------------

// Adjoints of a record's values.
template <typename R>
struct WallBar {
  R t[3], utan, G, tau;
};

// Vector-Jacobian product of the wall reconstruction collision (sigma = 0,
// modeled velocity v = u_tan t + (u.n) n, non-equilibrium -3 w rho tau G
// (c.t)(c.n), Guo source at v; third-order equilibrium with RR) in precision
// R, for the record held fixed: the adjoint of input population i goes to
// out(i, value); the adjoints of the record's values to rb.
// With Sfd (hybrid collision) the non-equilibrium is the full one,
// -3 w rho tau (c.S'.c - c_s^2 tr S') with S' = S + (e n^T + n e^T),
// e = (G/2) t - (S n - (n.S.n) n), and the adjoint of the finite-difference
// strain S goes to Sb.
template <int Q, typename R, bool RR, typename OUT>
__device__ __forceinline__ void wall_collide_vjp(const R g[Q], const R mu[Q], const R nv[3], const R tv[3], R utan,
                                                 R G, R tau, const KArgs &k, OUT out, WallBar<R> &rb,
                                                 const R *Sfd = nullptr, R *Sb = nullptr) {
  // ---- forward recomputation (as in the wall kernel)
  R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += g[i];
    acc(jx, Lat<Q>::c(i, 0), g[i]);
    acc(jy, Lat<Q>::c(i, 1), g[i]);
    acc(jz, Lat<Q>::c(i, 2), g[i]);
  }
  const R rho = R(1) + drho;
  const R Fx = R(k.F[0]), Fy = R(k.F[1]), Fz = R(k.F[2]);
  const R ir = R(1) / rho;
  const R ux = (jx + R(0.5) * Fx) * ir, uy = (jy + R(0.5) * Fy) * ir, uz = (jz + R(0.5) * Fz) * ir;
  const R nx = nv[0], ny = nv[1], nz = nv[2], tx = tv[0], ty = tv[1], tz = tv[2];
  const R un = ux * nx + uy * ny + uz * nz;
  const R vx = utan * tx + un * nx, vy = utan * ty + un * ny, vz = utan * tz + un * nz;
  const R vv = vx * vx + vy * vy + vz * vz;
  const R vF = vx * Fx + vy * Fy + vz * Fz;
  const R om = R(1) / tau;
  const R c1 = R(1) - om, c2 = R(1) - R(0.5) * om;
  const R fd = R(-3) * rho * tau * G;
  const bool full = Sfd != nullptr;
  const R hg = R(0.5) * G;
  R Sw[6] = {};
  if (full) {
    const R snx = Sfd[0] * nx + Sfd[3] * ny + Sfd[4] * nz;
    const R sny = Sfd[3] * nx + Sfd[1] * ny + Sfd[5] * nz;
    const R snz = Sfd[4] * nx + Sfd[5] * ny + Sfd[2] * nz;
    const R nSn = nx * snx + ny * sny + nz * snz;
    const R ex = hg * tx - (snx - nSn * nx), ey = hg * ty - (sny - nSn * ny), ez = hg * tz - (snz - nSn * nz);
    Sw[0] = Sfd[0] + R(2) * ex * nx;
    Sw[1] = Sfd[1] + R(2) * ey * ny;
    Sw[2] = Sfd[2] + R(2) * ez * nz;
    Sw[3] = Sfd[3] + ex * ny + nx * ey;
    Sw[4] = Sfd[4] + ex * nz + nx * ez;
    Sw[5] = Sfd[5] + ey * nz + ny * ez;
  }
  // ---- reverse through the outputs
  R s0 = R(0), s1 = R(0), stn = R(0), sg = R(0);
  R qxx = R(0), qyy = R(0), qzz = R(0), qxy = R(0), qxz = R(0), qyz = R(0);  // sum mu w c c
  R evx = R(0), evy = R(0), evz = R(0);  // sum mu w (3 + 9 c.v) c
  R gux = R(0), guy = R(0), guz = R(0);  // sum mu w 9 (c.F) c
  R snx = R(0), sny = R(0), snz = R(0);  // sum mu w (c.n) c
  R M[7];
#pragma unroll
  for (int m = 0; m < 7; ++m) M[m] = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = Lat<Q>::c(i, 0), cy = Lat<Q>::c(i, 1), cz = Lat<Q>::c(i, 2);
    const R mw = mu[i] * R(Lat<Q>::w(i));
    const R cv = dot3(cx, cy, cz, vx, vy, vz);
    const R ct = dot3(cx, cy, cz, tx, ty, tz);
    const R cn = dot3(cx, cy, cz, nx, ny, nz);
    const R cF = dot3(cx, cy, cz, Fx, Fy, Fz);
    s0 += mw;
    s1 += mw * (R(3) * cv + R(4.5) * cv * cv - R(1.5) * vv);
    stn += mw * ct * cn;
    sg += mw * (R(3) * (cF - vF) + R(9) * cv * cF);
    const R te = mw * (R(3) + R(9) * cv);
    acc(evx, cx, te);
    acc(evy, cy, te);
    acc(evz, cz, te);
    const R tg = mw * R(9) * cF;
    acc(gux, cx, tg);
    acc(guy, cy, tg);
    acc(guz, cz, tg);
    const R tn = mw * cn;
    acc(snx, cx, tn);
    acc(sny, cy, tn);
    acc(snz, cz, tn);
    acc(qxx, cx * cx, mw);
    acc(qyy, cy * cy, mw);
    acc(qzz, cz * cz, mw);
    acc(qxy, cx * cy, mw);
    acc(qxz, cx * cz, mw);
    acc(qyz, cy * cz, mw);
    if constexpr (RR) {
#pragma unroll
      for (int kk = 0; kk < H3Basis<Q>::n; ++kk) {
        const double pk = H3Basis<Q>::P(kk, i);
        if (pk != 0.0) M[kk] += mw * R(pk);
      }
    }
  }
  // full strain: sum_i mu_i w_i (c.S'.c - c_s^2 tr S') = W . S' (Z), with
  // W the derivative in the six components xx, yy, zz, xy, xz, yz
  R W[6] = {}, Z = R(0);
  if (full) {
    W[0] = qxx - s0 * R(1.0 / 3.0);
    W[1] = qyy - s0 * R(1.0 / 3.0);
    W[2] = qzz - s0 * R(1.0 / 3.0);
    W[3] = R(2) * qxy;
    W[4] = R(2) * qxz;
    W[5] = R(2) * qyz;
#pragma unroll
    for (int m = 0; m < 6; ++m) Z += W[m] * Sw[m];
  }
  // the non-equilibrium's sum: sum_i mu_i f^(1,FD)_i / (-3 rho tau)
  const R zs = full ? Z : G * stn;
  // equilibrium and Guo source: drho directly, rho, and v
  R drhob = s0;
  R rhob = s1 + c1 * R(-3) * tau * zs;
  R vxb = rho * (evx - R(3) * vx * s0) + c2 * (gux - R(3) * Fx * s0);
  R vyb = rho * (evy - R(3) * vy * s0) + c2 * (guy - R(3) * Fy * s0);
  R vzb = rho * (evz - R(3) * vz * s0) + c2 * (guz - R(3) * Fz * s0);
  if constexpr (RR) {
    // third-order equilibrium: rho v v v projected on the lattice's Hermite components
    constexpr H3Norms<Q> nrm = h3_norms<Q>();
    R Ab[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) Ab[m] = R(0);
#pragma unroll
    for (int kk = 0; kk < H3Basis<Q>::n; ++kk) {
      const R mk = M[kk] * R(1.0 / nrm.v[kk]);
      Ab[H3Basis<Q>::c0(kk)] += mk;
      if (H3Basis<Q>::sgn(kk) > 0.0) Ab[H3Basis<Q>::c1(kk)] += mk;
      if (H3Basis<Q>::sgn(kk) < 0.0) Ab[H3Basis<Q>::c1(kk)] -= mk;
    }
    // xxy, xxz, xyy, yyz, xzz, yzz, xyz
    rhob += Ab[0] * vx * vx * vy + Ab[1] * vx * vx * vz + Ab[2] * vx * vy * vy + Ab[3] * vy * vy * vz +
            Ab[4] * vx * vz * vz + Ab[5] * vy * vz * vz + Ab[6] * vx * vy * vz;
    vxb += rho * (Ab[0] * R(2) * vx * vy + Ab[1] * R(2) * vx * vz + Ab[2] * vy * vy + Ab[4] * vz * vz + Ab[6] * vy * vz);
    vyb += rho * (Ab[0] * vx * vx + Ab[2] * R(2) * vx * vy + Ab[3] * R(2) * vy * vz + Ab[5] * vz * vz + Ab[6] * vx * vz);
    vzb += rho * (Ab[1] * vx * vx + Ab[3] * vy * vy + Ab[4] * R(2) * vx * vz + Ab[5] * R(2) * vy * vz + Ab[6] * vx * vy);
  }
  // the record: c1 f^(1,FD) (with tau, and G and t through it) and v = u_tan t + un n
  rb.tau = zs * (R(-3) * rho * tau * om * om + c1 * R(-3) * rho) + sg * R(0.5) * om * om;
  rb.utan = vxb * tx + vyb * ty + vzb * tz;
  if (full) {
    // S' = S + e n^T + n e^T: to S directly and to e; e = (G/2) t - P S n, P = I - n n^T
    R Swb[6];
    const R cz = c1 * R(-3) * rho * tau;
#pragma unroll
    for (int m = 0; m < 6; ++m) Swb[m] = cz * W[m];
    const R ebx = R(2) * nx * Swb[0] + ny * Swb[3] + nz * Swb[4];
    const R eby = R(2) * ny * Swb[1] + nx * Swb[3] + nz * Swb[5];
    const R ebz = R(2) * nz * Swb[2] + nx * Swb[4] + ny * Swb[5];
    rb.G = R(0.5) * (tx * ebx + ty * eby + tz * ebz);
    rb.t[0] = hg * ebx + utan * vxb;
    rb.t[1] = hg * eby + utan * vyb;
    rb.t[2] = hg * ebz + utan * vzb;
    const R ne = nx * ebx + ny * eby + nz * ebz;
    const R sbx = -(ebx - ne * nx), sby = -(eby - ne * ny), sbz = -(ebz - ne * nz);  // adjoint of S n
    Sb[0] = Swb[0] + sbx * nx;
    Sb[1] = Swb[1] + sby * ny;
    Sb[2] = Swb[2] + sbz * nz;
    Sb[3] = Swb[3] + sbx * ny + sby * nx;
    Sb[4] = Swb[4] + sbx * nz + sbz * nx;
    Sb[5] = Swb[5] + sby * nz + sbz * ny;
  } else {
    rb.G = stn * c1 * R(-3) * rho * tau;
    rb.t[0] = c1 * fd * snx + utan * vxb;
    rb.t[1] = c1 * fd * sny + utan * vyb;
    rb.t[2] = c1 * fd * snz + utan * vzb;
  }
  // the cell's own velocity enters through un = u.n; u = (j + F/2)/rho
  const R unb = vxb * nx + vyb * ny + vzb * nz;
  const R uxb = unb * nx, uyb = unb * ny, uzb = unb * nz;
  rhob -= (uxb * ux + uyb * uy + uzb * uz) * ir;
  const R mxb = uxb * ir, myb = uyb * ir, mzb = uzb * ir;
  drhob += rhob;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    R v = drhob;
    acc(v, Lat<Q>::c(i, 0), mxb);
    acc(v, Lat<Q>::c(i, 1), myb);
    acc(v, Lat<Q>::c(i, 2), mzb);
    out(i, v);
  }
}

// Reverse of the record (FP64): from the adjoints of (t, u_tan, G, tau_b) to
// those of the reference cell's density and momentum j (u = (j + F/2)/rho),
// through t = u_t/|u_t|, the friction velocity (the root of g(U/u_tau) =
// y_r u_tau/nu, implicit derivative), u+_b (the root of g(u+) = y_b u_tau/nu,
// or U/u_tau when the reference is the wall cell itself), G(u_tau) and
// tau_b(G), and to the wall cell's C_S^2 (C2b) through G and tau_b.  An
// inactive record (|u_t| at or below 1e-300, or a failed solve) is constant:
// zero adjoint.
__device__ __forceinline__ void wall_record_vjp(const WallRec &w, const double u[3], double rho, const double n[3],
                                                double yr, double yb, bool self, double C2, const KArgs &k,
                                                const double tb[3], double utanb, double Gb, double taub,
                                                double &rhob, double jb[3], double &C2b) {
  rhob = 0.0;
  jb[0] = jb[1] = jb[2] = 0.0;
  C2b = 0.0;
  if (!w.active) return;
  const double nu = k.nu, inv_E = 1.0 / k.E, kap = k.kappa;
  const double ut = w.utau, U = w.U;
  const double Gt = Gb + 3.0 * C2 * taub;
  const double sq = sqrt(nu * nu + 4.0 * C2 * ut * ut);
  const double dG = 4.0 * ut / (nu + sq) - 8.0 * C2 * ut * ut * ut / (sq * (nu + sq) * (nu + sq));
  // G = 2 u_tau^2 / (nu + sq): dG/dC2 = -4 u_tau^4 / (sq (nu + sq)^2); tau_b = 3 (nu + C2 G) + 1/2
  C2b = 3.0 * w.G * taub - Gt * 4.0 * ut * ut * ut * ut / (sq * (nu + sq) * (nu + sq));
  double utb = Gt * dG, Ub = 0.0;
  if (self) {
    Ub = utanb;  // u_tan = u_tau (U / u_tau) = U
  } else {
    double gv, gdb;
    spalding_gd(w.uplus, kap, inv_E, gv, gdb);
    utb += utanb * (w.uplus + ut * (yb / nu) / gdb);
  }
  double gv, gdx;
  spalding_gd(U / ut, kap, inv_E, gv, gdx);
  Ub += utb * (gdx / ut) / (gdx * U / (ut * ut) + yr / nu);
  // u_t = u - (u.n) n, U = |u_t|, t = u_t / U
  const double tt = tb[0] * w.t[0] + tb[1] * w.t[1] + tb[2] * w.t[2];
  double a[3];
  for (int d = 0; d < 3; ++d) a[d] = Ub * w.t[d] + (tb[d] - tt * w.t[d]) / U;
  const double an = a[0] * n[0] + a[1] * n[1] + a[2] * n[2];
  for (int d = 0; d < 3; ++d) a[d] -= an * n[d];
  for (int d = 0; d < 3; ++d) jb[d] = a[d] / rho;
  rhob = -(a[0] * u[0] + a[1] * u[1] + a[2] * u[2]) / rho;
}

// Reverse step of the wall cells, one thread per record.  Reads the adjoint
// at the cell's write slots (common mode and deviations as in k_adjoint),
// recomputes the record from the reference cell's state, writes the cell's
// own adjoint and stores the reference cell's density and momentum adjoints
// in wadj[4][nwall].
template <int Q, typename S, bool ODD, bool RR, bool SEED, bool SLIP>
__global__ __launch_bounds__(256) void k_adjoint_wall(const S *__restrict__ pop, const uint8_t *__restrict__ flags,
                                                      typename Store<S>::R *__restrict__ dev,
                                                      const double *__restrict__ m_prev, double *__restrict__ m_next,
                                                      const int *__restrict__ wcell, const int *__restrict__ wref,
                                                      const double *__restrict__ rec, int nwall,
                                                      const uint64_t *__restrict__ wmask, double *__restrict__ wadj,
                                                      double *__restrict__ gcs, KArgs k, int p0, int p1,
                                                      const double *__restrict__ cnt, double sw,
                                                      typename Store<S>::R *__restrict__ sbar) {
  using R = typename Store<S>::R;
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwall) return;
  const int b = wcell[w], r = wref[w];
  int x, y, z;
  cell_xyz(b, k, x, y, z);
  const Nb n = make_nb(x, y, z, k);
  const LinkMask sm = wmask[w];  // precomputed from the static geometry
  const size_t N = (size_t)k.N;
  double scale = 1.0;
  if (x >= k.fringe_start) scale = 1.0 - (double)static_cast<const R *>(k.lam)[x];
  const double mx = m_prev[n.cell];
  const double d0 = (double)dev[write_slot<Q, ODD, SLIP>(n, sm, 0, N)];
  const double m = scale * (mx + d0);
  R dmu[Q];
  dmu[0] = R(0);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const double mw = m_prev[writer_of<Q, SLIP ? 2 : 1>(n, sm, i)];
    const double di = (double)dev[write_slot<Q, ODD, SLIP>(n, sm, i, N)];
    dmu[i] = (R)(scale * ((mw - mx) + (di - d0)));
  }
  R g[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) g[i] = Store<S>::ld(pop + read_slot<Q, ODD, SLIP>(n, sm, i, N));
  // the record, from the reference cell's state (the forward step's inputs)
  const size_t M = (size_t)nwall;
  double rho_r, ur[3];
  ref_velocity<Q, S, ODD, SLIP>(pop, wmask[M + w], r, k, rho_r, ur);
  const double nn[3] = {rec[WR_NX * M + w], rec[WR_NY * M + w], rec[WR_NZ * M + w]};
  const double yr = rec[WR_YR * M + w], yb = rec[WR_YB * M + w];
  const double C2 = cs2_of<R>(k, b);
  const WallRec wr = wall_record_of(ur, nn, yr, yb, r == b, C2, k);
  CellSeed cs{};
  if constexpr (SEED) cs = cell_seed<Q, R>(g, x, p0, p1, cnt, sw, k);
  const R nv[3] = {R(nn[0]), R(nn[1]), R(nn[2])};
  const R tv[3] = {R(wr.t[0]), R(wr.t[1]), R(wr.t[2])};
  WallBar<R> rb;
  auto store = [&](int i, R v) {
    if constexpr (SEED) v += (R)cs.template kin<Q>(i);
    dev[read_slot<Q, ODD, SLIP>(n, sm, i, N)] = v;
  };
  if (k.fdw > 0.0) {
    // hybrid collision: the full finite-difference strain (adjoint to sbar, for k_adjoint_fd)
    R Sfd[6], Sb[6];
    fd_strain<R>(n, k, Sfd);
    wall_collide_vjp<Q, R, RR>(g, dmu, nv, tv, R(wr.utan), R(wr.G), R(wr.tau), k, store, rb, Sfd, Sb);
#pragma unroll
    for (int m = 0; m < 6; ++m) sbar[(size_t)m * N + n.cell] = Sb[m];
  } else {
    wall_collide_vjp<Q, R, RR>(g, dmu, nv, tv, R(wr.utan), R(wr.G), R(wr.tau), k, store, rb);
  }
  m_next[n.cell] = SEED ? m + cs.base : m;
  const double tb[3] = {(double)rb.t[0], (double)rb.t[1], (double)rb.t[2]};
  double rhob, jb[3], C2b;
  wall_record_vjp(wr, ur, rho_r, nn, yr, yb, r == b, C2, k, tb, (double)rb.utan, (double)rb.G, (double)rb.tau, rhob,
                  jb, C2b);
  if (gcs) gcs[b] += C2b * 2.0 * cs_of<R>(k, b);
  wadj[w] = rhob;
  wadj[M + w] = jb[0];
  wadj[2 * M + w] = jb[1];
  wadj[3 * M + w] = jb[2];
}

// Adds the records' density and momentum adjoints to their reference cells'
// adjoints (population i of cell r: rho_bar + c_i . j_bar), one thread per
// distinct reference cell, summing its records in a fixed order.
template <int Q, typename S, bool ODD, bool SLIP>
__global__ __launch_bounds__(256) void k_adjoint_ref(const uint8_t *__restrict__ flags,
                                                     typename Store<S>::R *__restrict__ dev,
                                                     const int *__restrict__ rcell, const int *__restrict__ roff,
                                                     const int *__restrict__ rrec, int nref,
                                                     const double *__restrict__ wadj, int nwall, KArgs k) {
  using R = typename Store<S>::R;
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nref) return;
  const size_t M = (size_t)nwall;
  double a = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
  for (int j = roff[u]; j < roff[u + 1]; ++j) {
    const int w = rrec[j];
    a += wadj[w];
    ax += wadj[M + w];
    ay += wadj[2 * M + w];
    az += wadj[3 * M + w];
  }
  const int r = rcell[u];
  int x, y, z;
  cell_xyz(r, k, x, y, z);
  const Nb n = make_nb(x, y, z, k);
  LinkMask sm = 0;
  if (ODD && (flags[r] & FL_NEAR)) sm = solid_mask<Q, SLIP>(n, flags);
  const size_t N = (size_t)k.N;
  R cur[Q];  // all loads before any store (see k_adjoint_fd)
#pragma unroll
  for (int i = 0; i < Q; ++i) cur[i] = dev[read_slot<Q, ODD, SLIP>(n, sm, i, N)];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    double v = a;
    acc(v, Lat<Q>::c(i, 0), ax);
    acc(v, Lat<Q>::c(i, 1), ay);
    acc(v, Lat<Q>::c(i, 2), az);
    dev[read_slot<Q, ODD, SLIP>(n, sm, i, N)] = (R)((double)cur[i] + v);
  }
}

// Hybrid collision, second pass of the reverse step: the adjoints of the
// cells' finite-difference strains (sbar, written by the first pass) go back
// to the velocities their stencils read, and from the velocity
// u = (j + F/2)/rho of each cell to its populations, d u_b / d f_i =
// (c_ib - u_b) / rho.  One thread per fluid cell, gathering from the cell
// itself and its six axis neighbours: along axis a, a central difference
// 0.5 (u(z + e_a) - u(z - e_a)) sends +/- 0.5 of row a of the gradient's
// adjoint to the two neighbours, a one-sided one sends +/- 1 to the
// neighbour and to z.  Every fluid cell but the lid's took a strain.
template <int Q, typename S, bool ODD, int SOLID>
__global__ __launch_bounds__(ABLOCK) void k_adjoint_fd(const uint8_t *__restrict__ flags,
                                                       typename Store<S>::R *__restrict__ dev,
                                                       const typename Store<S>::R *__restrict__ sbar, KArgs k,
                                                       ATiles t) {
  using R = typename Store<S>::R;
  int x, y, z;
  if (!atile_xyz(k, t, x, y, z)) return;
  const Nb n = make_nb(x, y, z, k);
  const uint8_t fl = flags[n.cell];
  if (!(fl & FL_FLUID)) return;
  const size_t N = (size_t)k.N;
  auto fluid = [&](int c) { return (flags[c] & FL_FLUID) != 0; };
  auto strained = [&](int c) { return (flags[c] & (FL_FLUID | FL_LID)) == FL_FLUID; };
  // row a of the adjoint of D (D_ab = d_a u_b): S_aa = D_aa, S_ab = (D_ab + D_ba) / 2
  auto row = [&](int c, int a, R r[3]) {
    constexpr int idx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
#pragma unroll
    for (int b = 0; b < 3; ++b) r[b] = (a == b ? R(1) : R(0.5)) * sbar[(size_t)idx[a][b] * N + (size_t)c];
  };
  const int pos[3] = {x, y, z}, ext[3] = {k.nx, k.ny, k.nz};
  R ub[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R r[3];
    const bool hm = !((n.out >> (2 * a)) & 1u), hp = !((n.out >> (2 * a + 1)) & 1u);
    const int cm = n.cell + n.d[a][0], cp = n.cell + n.d[a][1];
    const bool fm = hm && fluid(cm), fp = hp && fluid(cp);
    // the cell's own strain: a one-sided difference reads its velocity
    if (fp != fm && strained(n.cell)) {
      row(n.cell, a, r);
      const R sg = fp ? R(-1) : R(1);
#pragma unroll
      for (int b = 0; b < 3; ++b) ub[b] += sg * r[b];
    }
    // the neighbour below along a (this cell is its upper neighbour)
    if (fm && strained(cm)) {
      int q[3] = {pos[0], pos[1], pos[2]};
      q[a] = pos[a] == 0 ? ext[a] - 1 : pos[a] - 1;
      const Nb nm = make_nb(q[0], q[1], q[2], k);
      const bool both = !((nm.out >> (2 * a)) & 1u) && fluid(cm + nm.d[a][0]);
      row(cm, a, r);
      const R wgt = both ? R(0.5) : R(1);
#pragma unroll
      for (int b = 0; b < 3; ++b) ub[b] += wgt * r[b];
    }
    // the neighbour above along a (this cell is its lower neighbour)
    if (fp && strained(cp)) {
      int q[3] = {pos[0], pos[1], pos[2]};
      q[a] = pos[a] == ext[a] - 1 ? 0 : pos[a] + 1;
      const Nb np = make_nb(q[0], q[1], q[2], k);
      const bool both = !((np.out >> (2 * a + 1)) & 1u) && fluid(cp + np.d[a][1]);
      row(cp, a, r);
      const R wgt = both ? R(0.5) : R(1);
#pragma unroll
      for (int b = 0; b < 3; ++b) ub[b] -= wgt * r[b];
    }
  }
  const V4<R> v = static_cast<const V4<R> *>(k.vel)[n.cell];
  const R ir = R(1) / v.w;
  const R base = -(ub[0] * v.x + ub[1] * v.y + ub[2] * v.z) * ir;
  LinkMask sm = 0;
  if (SOLID && ODD && (fl & FL_NEAR)) sm = solid_mask<Q, SOLID == 2>(n, flags);
  // all loads before any store: the slots are distinct, but the compiler
  // cannot know it and would otherwise wait for each load in turn
  R cur[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) cur[i] = dev[read_slot<Q, ODD, SOLID == 2>(n, sm, i, N)];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    R d = base;
    acc(d, Lat<Q>::c(i, 0), ub[0] * ir);
    acc(d, Lat<Q>::c(i, 1), ub[1] * ir);
    acc(d, Lat<Q>::c(i, 2), ub[2] * ir);
    dev[read_slot<Q, ODD, SOLID == 2>(n, sm, i, N)] = cur[i] + d;
  }
}

// Adjoint field = dJ/df of the current state for the terminal objective
// J = c_s^2 (<rho>_{x=p0} - <rho>_{x=p1}) + <rho |u|^2 / 2>; the fluid-cell
// counts come from the objective reduction already in cnt[0..2].
template <int Q, typename S, bool ODD, int SOLID>
__global__ __launch_bounds__(ABLOCK) void k_seed(const S *__restrict__ pop, const uint8_t *__restrict__ flags,
                                                 typename Store<S>::R *__restrict__ dev, double *__restrict__ m_cur, KArgs k,
                                                 ATiles t, int p0,
                                                 int p1, const double *__restrict__ cnt, double w) {
  int x, y, z;
  if (!atile_xyz(k, t, x, y, z)) return;
  const Nb n = make_nb(x, y, z, k);
  const uint8_t fl = flags[n.cell];
  if (!(fl & FL_FLUID)) return;
  LinkMask sm = 0;
  if (SOLID && ODD && (fl & FL_NEAR)) sm = solid_mask<Q, SOLID == 2>(n, flags);
  const size_t N = (size_t)k.N;
  double g[Q];
  double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    g[i] = (double)Store<S>::ld(pop + read_slot<Q, ODD, SOLID == 2>(n, sm, i, N));
    drho += g[i];
    acc(jx, Lat<Q>::c(i, 0), g[i]);
    acc(jy, Lat<Q>::c(i, 1), g[i]);
    acc(jz, Lat<Q>::c(i, 2), g[i]);
  }
  const double rho = 1.0 + drho;
  const double ux = (jx + 0.5 * k.F[0]) / rho, uy = (jy + 0.5 * k.F[1]) / rho, uz = (jz + 0.5 * k.F[2]) / rho;
  const double uu = ux * ux + uy * uy + uz * uz;
  double base = 0.0;
  if (x == p0) base += w / (3.0 * cnt[0]);
  if (x == p1) base -= w / (3.0 * cnt[1]);
  const double inf = w / cnt[2];
  using R = typename Store<S>::R;
  m_cur[n.cell] = base;  // common mode; the deviations carry the kinetic-energy part
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double cu = dot3(Lat<Q>::c(i, 0), Lat<Q>::c(i, 1), Lat<Q>::c(i, 2), ux, uy, uz);
    dev[read_slot<Q, ODD, SOLID == 2>(n, sm, i, N)] = (R)((cu - 0.5 * uu) * inf);
  }
}

// Natural order [q][N] (FP64 values) <-> in-memory form of the current
// parity (common mode + deviations; a cell's own read slots are its writes).
template <int Q, bool ODD, int SOLID, typename R>
__global__ __launch_bounds__(ABLOCK) void k_to_natural(const uint8_t *__restrict__ flags,
                                                       const double *__restrict__ m_cur,
                                                       const R *__restrict__ dev, double *__restrict__ nat,
                                                       KArgs k, ATiles t) {
  int x, y, z;
  if (!atile_xyz(k, t, x, y, z)) return;
  const Nb n = make_nb(x, y, z, k);
  const uint8_t fl = flags[n.cell];
  const size_t N = (size_t)k.N;
  if (!(fl & FL_FLUID)) {
#pragma unroll
    for (int i = 0; i < Q; ++i) nat[(size_t)i * N + n.cell] = 0.0;
    return;
  }
  LinkMask sm = 0;
  if (SOLID && ODD && (fl & FL_NEAR)) sm = solid_mask<Q, SOLID == 2>(n, flags);
  const double m = m_cur[n.cell];
#pragma unroll
  for (int i = 0; i < Q; ++i) nat[(size_t)i * N + n.cell] = m + (double)dev[read_slot<Q, ODD, SOLID == 2>(n, sm, i, N)];
}

template <int Q, bool ODD, int SOLID, typename R>
__global__ __launch_bounds__(ABLOCK) void k_from_natural(const uint8_t *__restrict__ flags,
                                                         const double *__restrict__ nat,
                                                         double *__restrict__ m_cur, R *__restrict__ dev,
                                                         KArgs k, ATiles t) {
  int x, y, z;
  if (!atile_xyz(k, t, x, y, z)) return;
  const Nb n = make_nb(x, y, z, k);
  const uint8_t fl = flags[n.cell];
  if (!(fl & FL_FLUID)) return;
  const size_t N = (size_t)k.N;
  LinkMask sm = 0;
  if (SOLID && ODD && (fl & FL_NEAR)) sm = solid_mask<Q, SOLID == 2>(n, flags);
  const double m = nat[n.cell];
  m_cur[n.cell] = m;
#pragma unroll
  for (int i = 0; i < Q; ++i) dev[read_slot<Q, ODD, SOLID == 2>(n, sm, i, N)] = (R)(nat[(size_t)i * N + n.cell] - m);
}

// ---------------------------------------------------------------------------
static int check(lbm_ctx *ctx, const char *what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? LBM_OK : hip_fail(ctx, e, what);
}

template <typename F>
static int adispatch(lbm_ctx *ctx, F &&f) {
  const bool odd = (ctx->steps & 1) != 0;
  auto by_geo = [&]<int Q, typename S>() {
    if (odd) {
      if (ctx->has_slip) return f.template operator()<Q, S, true, 2>();
      return ctx->has_solid ? f.template operator()<Q, S, true, 1>() : f.template operator()<Q, S, true, 0>();
    }
    if (ctx->has_slip) return f.template operator()<Q, S, false, 2>();
    return ctx->has_solid ? f.template operator()<Q, S, false, 1>() : f.template operator()<Q, S, false, 0>();
  };
  if (ctx->q == 19) {
    if (ctx->p.storage == LBM_F64) return by_geo.template operator()<19, double>();
    if (ctx->p.storage == LBM_F32DEV) return by_geo.template operator()<19, float>();
    return by_geo.template operator()<19, _Float16>();
  }
  if (ctx->p.storage == LBM_F64) return by_geo.template operator()<27, double>();
  if (ctx->p.storage == LBM_F32DEV) return by_geo.template operator()<27, float>();
  return by_geo.template operator()<27, _Float16>();
}

// Pointers into an adjoint buffer: the common-mode arrays of the current
// and the other parity, and the deviations.
struct AdjPtrs {
  double *m_cur, *m_other;
  void *dev;
  double *wadj;  // [4][nwall] (wall model)
  void *sbar;    // [6][N] compute type (hybrid collision)
};
static AdjPtrs adj_ptrs(lbm_ctx *ctx, void *lamv) {
  const bool fd = ctx->ka.fdw > 0.0;
  const AdjLayout L = adj_layout(ctx->N, ctx->q, ctx->p.storage == LBM_F64 ? 8 : 4, ctx->nwall, fd);
  double *m0 = (double *)lamv, *m1 = m0 + ctx->N;
  const bool odd = (ctx->steps & 1) != 0;
  return {odd ? m1 : m0, odd ? m0 : m1, (char *)lamv + L.d_off,
          ctx->nwall > 0 ? (double *)((char *)lamv + L.wadj_off) : nullptr,
          fd ? (void *)((char *)lamv + L.sbar_off) : nullptr};
}

// The reverse step for one lattice and storage type.  Its kernels are many
// (parity, geometry, porosity, collision model, seeds, open faces) and heavy,
// so the build compiles this file once more per (Q, S) pair with ADJ_PART set,
// each copy instantiating one pair; the main copy dispatches to them.
template <int Q, typename S>
int adjoint_step_qs(lbm_ctx *ctx, void *lamv, void *gradv, void *gcsv, double seed_w, const int *planes) {
  const ATiles t = atiles_of(ctx->ka);
  const AdjPtrs a = adj_ptrs(ctx, lamv);
  auto body = [&]<bool ODD, int SOLID>() {
    using R = typename Store<S>::R;
    R *dev = (R *)a.dev;
    double *grad = (double *)gradv;
    double *gcs = (double *)gcsv;
    const R *phi = (const R *)ctx->phi;
    // reads the common modes of the later state (the other parity), writes this parity's
    const int p0 = planes ? planes[0] : 0, p1 = planes ? planes[1] : 0;
    const double *cnt = ctx->result + 8 + 3;  // fluid-cell counts of the last objective evaluation
    R *sbar = (R *)a.sbar;
    const bool hyb = ctx->ka.fdw > 0.0;
    if (hyb) {
      // the hybrid's velocity field of the state this step reads
      const int rc = dev_velocity4(ctx);
      if (rc != LBM_OK) return rc;
    }
    auto go = [&](auto kern) {
      kern<<<t.nblocks, ABLOCK, 0, ctx->stream>>>((const S *)ctx->pop, ctx->flags, dev, a.m_other, a.m_cur, phi,
                                                  grad, gcs, ctx->ka, t, p0, p1, cnt, seed_w, sbar);
    };
    auto by_seed = [&]<bool POROUS, bool RR>() {
      if constexpr (RR) {
        // the hybrid collision (never with open faces)
        if (hyb) {
          if (seed_w != 0.0) go(k_adjoint<Q, S, ODD, POROUS, SOLID, true, true, false, true>);
          else go(k_adjoint<Q, S, ODD, POROUS, SOLID, true, false, false, true>);
          return;
        }
      }
      // open x faces make x non-periodic, so their domains always have solid links
      if constexpr (SOLID) {
        if (ctx->has_open) {
          if (seed_w != 0.0) go(k_adjoint<Q, S, ODD, POROUS, SOLID, RR, true, true>);
          else go(k_adjoint<Q, S, ODD, POROUS, SOLID, RR, false, true>);
          return;
        }
      }
      if (seed_w != 0.0) go(k_adjoint<Q, S, ODD, POROUS, SOLID, RR, true>);
      else go(k_adjoint<Q, S, ODD, POROUS, SOLID, RR, false>);
    };
    if (ctx->porous) {
      if (ctx->ka.rr) by_seed.template operator()<true, true>();
      else by_seed.template operator()<true, false>();
    } else {
      if (ctx->ka.rr) by_seed.template operator()<false, true>();
      else by_seed.template operator()<false, false>();
    }
    int rc = check(ctx, "k_adjoint");
    // the strains' adjoints to the velocities, once every cell has written its own
    auto fd_pass = [&]() -> int {
      if (!hyb) return LBM_OK;
      k_adjoint_fd<Q, S, ODD, SOLID><<<t.nblocks, ABLOCK, 0, ctx->stream>>>(ctx->flags, dev, sbar, ctx->ka, t);
      return check(ctx, "k_adjoint_fd");
    };
    if (rc != LBM_OK) return rc;
    if (ctx->nwall == 0) return fd_pass();
    if constexpr (SOLID) {
      // wall cells, then their contributions to the reference cells
      const int nw = ctx->nwall, wb = (nw + 255) / 256;
      auto gow = [&](auto kern) {
        kern<<<wb, 256, 0, ctx->stream>>>((const S *)ctx->pop, ctx->flags, dev, a.m_other, a.m_cur, ctx->wcell,
                                         ctx->wref, ctx->wrec, nw, ctx->wmask, a.wadj, gcs, ctx->ka, p0, p1, cnt,
                                         seed_w, sbar);
      };
      constexpr bool SLIP = SOLID == 2;
      if (ctx->ka.rr) {
        if (seed_w != 0.0) gow(k_adjoint_wall<Q, S, ODD, true, true, SLIP>);
        else gow(k_adjoint_wall<Q, S, ODD, true, false, SLIP>);
      } else {
        if (seed_w != 0.0) gow(k_adjoint_wall<Q, S, ODD, false, true, SLIP>);
        else gow(k_adjoint_wall<Q, S, ODD, false, false, SLIP>);
      }
      rc = check(ctx, "k_adjoint_wall");
      if (rc != LBM_OK) return rc;
      const int rb = (ctx->nref + 255) / 256;
      k_adjoint_ref<Q, S, ODD, SLIP><<<rb, 256, 0, ctx->stream>>>(ctx->flags, dev, ctx->wref_cell, ctx->wref_off,
                                                          ctx->wref_rec, ctx->nref, a.wadj, nw, ctx->ka);
      rc = check(ctx, "k_adjoint_ref");
      if (rc != LBM_OK) return rc;
      return fd_pass();
    }
    return rc;
  };
  const bool odd = (ctx->steps & 1) != 0;
  if (odd) {
    if (ctx->has_slip) return body.template operator()<true, 2>();
    return ctx->has_solid ? body.template operator()<true, 1>() : body.template operator()<true, 0>();
  }
  if (ctx->has_slip) return body.template operator()<false, 2>();
  return ctx->has_solid ? body.template operator()<false, 1>() : body.template operator()<false, 0>();
}

#define LBM_ADJ_PAIRS(X) X(19, double) X(19, float) X(19, _Float16) X(27, double) X(27, float) X(27, _Float16)
#define LBM_ADJ_DECL(Q, S) \
  template int adjoint_step_qs<Q, S>(lbm_ctx *, void *, void *, void *, double, const int *);
#define LBM_ADJ_EXTERN(Q, S) \
  extern template int adjoint_step_qs<Q, S>(lbm_ctx *, void *, void *, void *, double, const int *);

#if defined(ADJ_PART)
// one (Q, S) pair per part
#if ADJ_PART == 0
LBM_ADJ_DECL(19, double)
#elif ADJ_PART == 1
LBM_ADJ_DECL(19, float)
#elif ADJ_PART == 2
LBM_ADJ_DECL(19, _Float16)
#elif ADJ_PART == 3
LBM_ADJ_DECL(27, double)
#elif ADJ_PART == 4
LBM_ADJ_DECL(27, float)
#elif ADJ_PART == 5
LBM_ADJ_DECL(27, _Float16)
#endif
#else
LBM_ADJ_PAIRS(LBM_ADJ_EXTERN)

int dev_adjoint_step(lbm_ctx *ctx, void *lamv, void *gradv, void *gcsv, double seed_w, const int *planes) {
  if (ctx->q == 19) {
    if (ctx->p.storage == LBM_F64) return adjoint_step_qs<19, double>(ctx, lamv, gradv, gcsv, seed_w, planes);
    if (ctx->p.storage == LBM_F32DEV) return adjoint_step_qs<19, float>(ctx, lamv, gradv, gcsv, seed_w, planes);
    return adjoint_step_qs<19, _Float16>(ctx, lamv, gradv, gcsv, seed_w, planes);
  }
  if (ctx->p.storage == LBM_F64) return adjoint_step_qs<27, double>(ctx, lamv, gradv, gcsv, seed_w, planes);
  if (ctx->p.storage == LBM_F32DEV) return adjoint_step_qs<27, float>(ctx, lamv, gradv, gcsv, seed_w, planes);
  return adjoint_step_qs<27, _Float16>(ctx, lamv, gradv, gcsv, seed_w, planes);
}

int dev_adjoint_seed(lbm_ctx *ctx, const int planes[2], void *lamv, double w) {
  int rc = dev_objective(ctx, planes);  // fills the fluid-cell counts
  if (rc != LBM_OK) return rc;
  const ATiles t = atiles_of(ctx->ka);
  const AdjPtrs a = adj_ptrs(ctx, lamv);
  return adispatch(ctx, [&]<int Q, typename S, bool ODD, int SOLID>() {
    using R = typename Store<S>::R;
    k_seed<Q, S, ODD, SOLID><<<t.nblocks, ABLOCK, 0, ctx->stream>>>((const S *)ctx->pop, ctx->flags, (R *)a.dev,
                                                                   a.m_cur, ctx->ka, t, planes[0], planes[1],
                                                                   ctx->result + 8 + 3, w);
    return check(ctx, "k_seed");
  });
}

int dev_layout_to_natural(lbm_ctx *ctx, const void *lamv, void *natv) {
  const ATiles t = atiles_of(ctx->ka);
  const AdjPtrs a = adj_ptrs(ctx, const_cast<void *>(lamv));
  return adispatch(ctx, [&]<int Q, typename S, bool ODD, int SOLID>() {
    using R = typename Store<S>::R;
    k_to_natural<Q, ODD, SOLID, R><<<t.nblocks, ABLOCK, 0, ctx->stream>>>(ctx->flags, a.m_cur, (const R *)a.dev,
                                                                         (double *)natv, ctx->ka, t);
    return check(ctx, "k_to_natural");
  });
}

int dev_layout_from_natural(lbm_ctx *ctx, const void *natv, void *lamv) {
  const ATiles t = atiles_of(ctx->ka);
  const AdjPtrs a = adj_ptrs(ctx, lamv);
  return adispatch(ctx, [&]<int Q, typename S, bool ODD, int SOLID>() {
    using R = typename Store<S>::R;
    k_from_natural<Q, ODD, SOLID, R><<<t.nblocks, ABLOCK, 0, ctx->stream>>>(ctx->flags, (const double *)natv,
                                                                           a.m_cur, (R *)a.dev, ctx->ka, t);
    return check(ctx, "k_from_natural");
  });
}

#endif  // ADJ_PART

}  // namespace lbmk
