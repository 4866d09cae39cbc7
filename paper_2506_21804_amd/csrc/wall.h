// Wall record of the Spalding wall model (Sec. 2.2.1, Eqs. (15)-(17)), FP64,
// shared by the forward wall kernels and the reverse step: the friction
// velocity at the reference cell, the modeled tangential speed at the wall
// cell, the modeled strain and the wall cell's relaxation time, plus the
// intermediates the reverse step differentiates through.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"
#include "lattice.h"

namespace lbmk {

// Spalding function g(u+) = u+ + R4(kappa u+)/E with R_m(a) = exp(a) -
// sum_{n<m} a^n/n!, and g'(u+) = 1 + kappa R3(kappa u+)/E.  Below a = 1/2
// the remainders are summed as their power series (no cancellation), by
// Horner over 24 terms with reciprocal factorials as compile-time constants.
__host__ __device__ constexpr double inv_factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return 1.0 / f;
}
template <int M>
__device__ __forceinline__ double exp_tail(double a) {
  double p = inv_factorial(M + 23);
#pragma unroll
  for (int n = M + 22; n >= M; --n) p = fma(p, a, inv_factorial(n));
  double am = a;
#pragma unroll
  for (int n = 1; n < M; ++n) am *= a;
  return p * am;
}
// g and g' at u+ (one exponential for both); inv_E = 1/E.
__device__ __forceinline__ void spalding_gd(double up, double kappa, double inv_E, double &g, double &gd) {
  const double a = kappa * up;
  double r3, r4;
  if (a >= 0.0 && a < 0.5) {
    r4 = exp_tail<4>(a);
    r3 = exp_tail<3>(a);
  } else {
    r3 = exp(a) - 1.0 - a - 0.5 * a * a;
    r4 = r3 - a * a * a * (1.0 / 6.0);
  }
  g = up + r4 * inv_E;
  gd = 1.0 + kappa * r3 * inv_E;
}

// Density and Guo velocity u = (j + F/2)/rho of cell r's current state, FP64.
// rmask: the cell's link mask, precomputed (0 unless it has a solid link).
template <int Q, typename S, bool ODD, bool SLIP>
__device__ __forceinline__ void ref_velocity(const S *__restrict__ pop, LinkMask rmask, int r, const KArgs &k,
                                             double &rho, double u[3]) {
  int x, y, z;
  cell_xyz(r, k, x, y, z);
  const Nb n = make_nb(x, y, z, k);
  const LinkMask sm = ODD ? rmask : 0u;
  const size_t N = (size_t)k.N;
  double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double gi = (double)Store<S>::ld(pop + read_slot<Q, ODD, SLIP>(n, sm, i, N));
    drho += gi;
    acc(jx, Lat<Q>::c(i, 0), gi);
    acc(jy, Lat<Q>::c(i, 1), gi);
    acc(jz, Lat<Q>::c(i, 2), gi);
  }
  rho = 1.0 + drho;
  u[0] = (jx + 0.5 * k.F[0]) / rho;
  u[1] = (jy + 0.5 * k.F[1]) / rho;
  u[2] = (jz + 0.5 * k.F[2]) / rho;
}

struct WallRec {
  double t[3], utan, G, tau, utau;
  double U, uplus;  // |u_t| at the reference cell, u+ at the wall cell
  bool active;      // U > 1e-300 and both solves converged (otherwise the record is zero)
  bool fail;        // a Newton solve failed
};

// The record from the reference cell's velocity u and the unit normal n;
// yr, yb the wall distances of the reference and the wall cell; self: the
// reference cell is the wall cell itself (u+_b = U/u_tau); C2 the wall cell's
// C_S^2.
__device__ __forceinline__ WallRec wall_record_of(const double u[3], const double n[3], double yr, double yb,
                                                  bool self, double C2, const KArgs &k) {
  WallRec w;
  const double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
  const double tx = u[0] - un * n[0], ty = u[1] - un * n[1], tz = u[2] - un * n[2];
  const double U = sqrt(tx * tx + ty * ty + tz * tz);
  const double nu = k.nu, kap = k.kappa, E = k.E;
  w.utau = 0.0;
  w.utan = 0.0;
  w.G = 0.0;
  w.tau = 3.0 * nu + 0.5;
  w.t[0] = w.t[1] = w.t[2] = 0.0;
  w.U = U;
  w.uplus = 0.0;
  w.active = false;
  w.fail = false;
  if (U > 1e-300) {
    // F(u) = g(U/u) - yr u / nu is convex and decreasing in u, and the
    // laminar value ulam = sqrt(nu U / yr) is a lower bound of its root.  From
    // any start, the first Newton step lands at or below the root; clamping
    // every iterate to ulam keeps it in range, and from there the iterates
    // climb monotonically.  The start is the log-law friction velocity (two
    // fixed-point steps of u = kappa U / ln(E yr u / nu) from ulam), within a
    // few per cent of the root: at y+ of 100-250 Newton then needs about 5
    // iterations instead of 17-29 from ulam.  The root is the same.
    const double ulam = sqrt(nu * U / yr);
    double ut = ulam;
    for (int j = 0; j < 2; ++j) {
      const double L = log(E * yr * ut / nu);
      if (L > 1.0) ut = fmax(ulam, kap * U / L);
    }
    bool conv = false;
    const double inv_E = 1.0 / E, a_r = yr / nu;  // F(u) = g(U/u) - a_r u
    if (kap * U / ulam <= 700.0) {
      for (int it = 0; it < 100; ++it) {
        const double iu = 1.0 / ut;
        const double xx = U * iu;
        double gv, gdv;
        spalding_gd(xx, kap, inv_E, gv, gdv);
        const double Fv = gv - a_r * ut;
        const double dF = -gdv * xx * iu - a_r;
        const double st = -Fv / dF;
        ut = fmax(ut + st, ulam);
        if (fabs(st) <= 1e-15 * ut) {
          conv = true;
          break;
        }
      }
    }
    double up = U / ut;
    if (conv && !self) {
      // u+ at the wall cell: g(u+) = y+_b by Newton from an upper bound of
      // the root (g convex increasing: the iterates decrease monotonically).
      const double ypb = yb * ut / nu;
      const double K = kap * ypb;
      double s = fmin(ypb, log(E * ypb + 1.0 + K + 0.5 * K * K + K * K * K / 6.0) / kap);
      if (yr >= yb) s = fmin(s, up);
      conv = false;
      if (kap * s <= 700.0) {
        for (int it = 0; it < 100; ++it) {
          double gv, gdv;
          spalding_gd(s, kap, inv_E, gv, gdv);
          const double st = -(gv - ypb) / gdv;
          s += st;
          if (fabs(st) <= 1e-15 * fabs(s)) {
            conv = true;
            break;
          }
        }
      }
      up = s;
    }
    if (!conv) {
      w.fail = true;
    } else {
      w.active = true;
      w.utau = ut;
      w.uplus = up;
      w.utan = ut * up;
      w.t[0] = tx / U;
      w.t[1] = ty / U;
      w.t[2] = tz / U;
      w.G = 2.0 * ut * ut / (nu + sqrt(nu * nu + 4.0 * C2 * ut * ut));
      w.tau = 3.0 * (nu + C2 * w.G) + 0.5;
    }
  }
  return w;
}

}  // namespace lbmk
