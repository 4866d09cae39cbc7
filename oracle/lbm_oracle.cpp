/*
 * FP64 CPU oracle of the wall-modeled LBM-LES time step of Kummerlaender,
 * Bukreev, Shimojima, Ito, Krause, "Large-Scale Simulations of Turbulent
 * Flows using Lattice Boltzmann Methods on Heterogeneous High Performance
 * Computers" (arXiv 2506.21804).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header or table with the HIP path.
 *
 * It is deliberately plain: two population lattices (f, f*), one cell at a
 * time, double precision, collide everything, then pull-stream everything.
 * No blocking, no fusion, no in-place tricks.  The scalar type is a template
 * parameter so the same code also runs on forward-mode dual numbers, which
 * gives exact directional derivatives (the "tangent" oracle of the adjoint).
 *
 * What one step computes (n -> n+1), in this order:
 *   1. wall prepass: for every wall-modeled cell b, friction velocity u_tau
 *      from the Spalding law (Sec. 2.2.1, Eqs. (15)-(17)) solved by Newton
 *      in FP64 at a reference cell r, the modeled tangential velocity at b
 *      and the modeled strain magnitude G;
 *   2. collision of every fluid cell: the homogenized LB update
 *      (Sec. 2.2, Eq. (6)) in its BGK form, with the Smagorinsky effective
 *      relaxation time (Eqs. (3),(4),(14)), the homogenized velocity
 *      (Eq. (12)), and Guo forcing; wall cells use the wall-model
 *      reconstruction (sigma = 0, solid velocity = modeled velocity,
 *      Sec. 2.2.1 last paragraph, non-equilibrium from Eq. (10));
 *      then the fringe blend / lid of the open-boundary urban setup;
 *   3. streaming with halfway bounce-back at solid links, and specular
 *      reflection at full-slip box faces (the outer walls of the
 *      street-canyon setup, Sec. 3.2).
 *
 * Readings of the paper where it is silent or garbled (each is also listed
 * in the design document):
 *   - lattice units, dx = dt = 1, c_s^2 = 1/3;
 *   - collision 0: second-order equilibrium (BGK); collision 1: the
 *     recursive regularized collision of Sec. 2.2 with sigma = 1 (Eqs. (6),
 *     (8), (9), (11)): third-order equilibrium, f^(1) rebuilt from its
 *     Hermite coefficients of order 1 (sum xi f^(1), which the Guo velocity
 *     makes -F/2), 2 (Pi^neq) and 3 (by the recursion u_a Pi_bc + u_b Pi_ac
 *     + u_c Pi_ab), each third-order term projected on the Hermite
 *     components the lattice carries (see hermite3 below);
 *   - hybrid collision (Eq. (7)) with weight fd_weight = 1 - sigma of the
 *     finite-difference strain: S^FD from central differences of the
 *     pre-collision velocity field of the same step (one-sided next to a
 *     non-fluid neighbour, zero with none), f^(1,FD) = -(w rho tau / c_s^2)
 *     H^(2) : S^FD; the hybrid blends the second-order part, the third-order
 *     part keeps the factor sigma and the first-order part (-F/2) is kept
 *     whole; wall cells (sigma = 0 there) use the full S^FD with its
 *     wall-normal shear replaced by the wall law's, G/2 along t;
 *   - f^(1) = f - f^eq(rho, u); f* = f^eq(rho, u_hat) + (1 - 1/tau)(f - f^eq(rho,u));
 *   - porosity phi in [0,1], 1 = fluid: u_hat = phi*u + (1-phi)*u_B, u_B = 0
 *     in the bulk (the weights of Eq. (12) read with d := 1 - phi);
 *   - tau_eff is the positive root of tau^2 - tau0*tau - C_S^2 |Pi| /
 *     (sqrt(2) rho c_s^4) = 0, i.e. nu_eff = nu0 + C_S^2 |S|, |S| = sqrt(2 S:S),
 *     with S taken from Pi^neq = -2 rho c_s^2 tau_eff S;
 *   - Eq. (10) read as f^(1,FD)_i = -(w_i rho tau / c_s^2) H^(2)_i : S;
 *   - Guo forcing, u = (j + F/2)/rho, source (1 - 1/(2 tau)) w_i
 *     [3(xi_i - u) + 9 (xi_i.u) xi_i].F;
 *   - smooth-wall Spalding constants kappa, E are parameters (0.41, 9.0);
 *   - wall cells: fluid cells with at least one solid link; normal from the
 *     sum of the solid links; reference cell one lattice step along the
 *     direction best aligned with the normal; stress-consistent strain
 *     G = 2 u_tau^2 / (nu + sqrt(nu^2 + 4 C_S^2 u_tau^2));
 *   - open x faces (open_x = 1; Sec. 2.2.2 imposes the inflow with a
 *     regularized local velocity condition, Sec. 3.2 closes the outlet with a
 *     fixed local pressure condition): the fluid cells of the planes x = 0
 *     (inlet) and x = nx - 1 (outlet) that are not lid cells replace their
 *     pre-collision populations before the collision.  The populations that
 *     enter through the face are unknown.  Inlet: u = (u_in(z), 0, 0), plus
 *     the vortex method's in-plane perturbation when vortices are set (the
 *     streamwise Langevin term, garbled in the paper, is left out),
 *     prescribed, rho from the known populations and u.n, and (regularized)
 *     the non-equilibrium of an unknown population is that of its opposite
 *     (known) one, Pi^neq is summed over all of them, and the cell's
 *     populations become f^eq(rho, u) + w H^(2) : Pi^neq / (2 c_s^4).
 *     Outlet: rho = rho_out prescribed, the normal velocity from the known
 *     populations, the tangential velocity zero, and the populations become
 *     f^eq(rho_out, u) (no non-equilibrium: rebuilt from the arriving
 *     populations it makes the outlet unstable as tau approaches 1/2).  The
 *     ordinary bulk collision follows.  These cells are never
 *     wall-modeled, links through an open face are otherwise handled like
 *     solid links, the outlet plane is left out of the fringe, and the body
 *     force must be zero.
 */
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <string>
#include <type_traits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {
/* The oracle's own parameter block (plain C layout for ctypes). */
typedef struct {
  int q, nx, ny, nz;
  int periodic[3];
  double tau0, cs_smag;
  double force[3];
  int wall_model;
  double kappa, E;
  int fringe_len;
  double u_ref, z0;
  int lid;
  int collision; /* 0: BGK (second-order equilibrium); 1: recursive regularized, third order */
  double fd_weight; /* 1 - sigma of Eq. (7): weight of the finite-difference strain (collision 1 only) */
  int open_x;       /* 1: velocity inlet at x = 0 and pressure outlet at x = nx - 1 (non-periodic x) */
  double rho_out;   /* density imposed at the outlet (open_x only) */
  int slip;         /* full-slip box faces: bit 2a the low face of axis a, bit 2a+1 the high face */
} orc_params;
}

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENONFINITE = -3, ORC_ENEWTON = -4 };

namespace {

/* ------------------------------------------------------------------------ */
/* Forward-mode dual number: value and one directional derivative.           */
/* ------------------------------------------------------------------------ */
struct Dual {
  double v, d;
  Dual(double v_ = 0.0, double d_ = 0.0) : v(v_), d(d_) {}
  Dual& operator+=(const Dual& b) { v += b.v; d += b.d; return *this; }
  Dual& operator-=(const Dual& b) { v -= b.v; d -= b.d; return *this; }
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
/* d sqrt(x) = dx / (2 sqrt(x)); at x = 0 the derivative is taken as 0 (the
 * subgradient convention for the Frobenius norm of a vanishing stress). */
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, s > 0.0 ? a.d / (2.0 * s) : 0.0);
}
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double der(double) { return 0.0; }
inline double der(const Dual& x) { return x.d; }
using std::sqrt;

/* ------------------------------------------------------------------------ */
/* Velocity sets.  D3Q19 is the stencil of the paper (Sec. 2.2, Fig. of the  */
/* lattice); D3Q27 adds the eight corner directions.  Ordering: rest, the    */
/* nine "positive" directions, (D3Q27: four corners with +x), then all       */
/* negatives in the same order.                                              */
/* ------------------------------------------------------------------------ */
struct VelSet {
  int q = 0;
  int c[27][3];
  double w[27];
  int opp[27];
};

VelSet make_velocity_set(int q) {
  VelSet v;
  v.q = q;
  static const int pos9[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0},
                                 {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};
  static const int corner4[4][3] = {{1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
  int npos = (q == 19) ? 9 : 13;
  for (int a = 0; a < 3; ++a) v.c[0][a] = 0;
  for (int k = 0; k < npos; ++k) {
    const int* e = (k < 9) ? pos9[k] : corner4[k - 9];
    for (int a = 0; a < 3; ++a) {
      v.c[1 + k][a] = e[a];
      v.c[1 + npos + k][a] = -e[a];
    }
  }
  for (int i = 0; i < q; ++i) {
    int n2 = v.c[i][0] * v.c[i][0] + v.c[i][1] * v.c[i][1] + v.c[i][2] * v.c[i][2];
    if (q == 19) {
      v.w[i] = (n2 == 0) ? 1.0 / 3.0 : (n2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
    } else {
      v.w[i] = (n2 == 0) ? 8.0 / 27.0 : (n2 == 1) ? 2.0 / 27.0 : (n2 == 2) ? 1.0 / 54.0 : 1.0 / 216.0;
    }
    for (int j = 0; j < q; ++j)
      if (v.c[j][0] == -v.c[i][0] && v.c[j][1] == -v.c[i][1] && v.c[j][2] == -v.c[i][2]) v.opp[i] = j;
  }
  return v;
}

/* Second-order equilibrium: w_i rho [1 + 3 xi.v + 9/2 (xi.v)^2 - 3/2 v.v]
 * (the Hermite equilibrium of Sec. 2.2 truncated after H^(2), c_s^2 = 1/3). */
template <class T>
void equilibrium(const VelSet& vs, const T& rho, const T v[3], T* feq) {
  T vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  for (int i = 0; i < vs.q; ++i) {
    T cv = double(vs.c[i][0]) * v[0] + double(vs.c[i][1]) * v[1] + double(vs.c[i][2]) * v[2];
    feq[i] = vs.w[i] * rho * (1.0 + 3.0 * cv + 4.5 * cv * cv - 1.5 * vv);
  }
}

/* ------------------------------------------------------------------------ */
/* Third-order Hermite terms of the recursive regularized collision         */
/* (Sec. 2.2, Eqs. (8), (9), (11)).                                          */
/*   H^(3)_abc(xi) = xi_a xi_b xi_c - c_s^2 (xi_a d_bc + xi_b d_ac + xi_c d_ab) */
/* Only components the lattice can carry enter.  On D3Q27 these are the six  */
/* of type xxy and xyz, mutually orthogonal in the weighted lattice sum      */
/* sum_i w_i P_i Q_i (xxx vanishes: xi^3 = xi).  On D3Q19 xyz vanishes too,   */
/* and the pairs (xxy, yzz), (xzz, xyy), (yyz, xxz) are not orthogonal there, */
/* so their sums and differences form the basis.  A symmetric third-order     */
/* tensor A enters as its orthogonal projection on that basis,               */
/*   w_i sum_P P_i <A, P> / (sum_j w_j P_j^2),  <A, P> = sum of A over the    */
/* components of P with their signs,                                         */
/* so that every admissible third moment sum_i P_i out_i equals <A, P>.       */
/* The norms come from the lattice itself, not from the continuous Hermite    */
/* norms (on D3Q19 they differ).                                             */
/* ------------------------------------------------------------------------ */
double hermite3(const VelSet& vs, int i, int a, int b, int c) {
  const double cs2 = 1.0 / 3.0;
  double xa = vs.c[i][a], xb = vs.c[i][b], xc = vs.c[i][c];
  return xa * xb * xc - cs2 * (xa * (b == c) + xb * (a == c) + xc * (a == b));
}

struct H3Basis {
  int n = 0;
  int ncomp[7];
  int comp[7][2][3];
  double sgn[7][2];
  double P[7][27];
  double norm[7];
};

H3Basis make_h3_basis(const VelSet& vs) {
  enum { X = 0, Y = 1, Z = 2 };
  H3Basis B;
  auto add = [&](std::initializer_list<int> t1, std::initializer_list<int> t2, double s2) {
    int k = B.n++;
    const int* a = t1.begin();
    for (int m = 0; m < 3; ++m) B.comp[k][0][m] = a[m];
    B.sgn[k][0] = 1.0;
    B.ncomp[k] = 1;
    if (t2.size() == 3) {
      const int* b = t2.begin();
      for (int m = 0; m < 3; ++m) B.comp[k][1][m] = b[m];
      B.sgn[k][1] = s2;
      B.ncomp[k] = 2;
    }
  };
  if (vs.q == 27) {
    add({X, X, Y}, {}, 0.0);
    add({X, X, Z}, {}, 0.0);
    add({X, Y, Y}, {}, 0.0);
    add({Y, Y, Z}, {}, 0.0);
    add({X, Z, Z}, {}, 0.0);
    add({Y, Z, Z}, {}, 0.0);
    add({X, Y, Z}, {}, 0.0);
  } else {
    add({X, X, Y}, {Y, Z, Z}, 1.0);
    add({X, X, Y}, {Y, Z, Z}, -1.0);
    add({X, Z, Z}, {X, Y, Y}, 1.0);
    add({X, Z, Z}, {X, Y, Y}, -1.0);
    add({Y, Y, Z}, {X, X, Z}, 1.0);
    add({Y, Y, Z}, {X, X, Z}, -1.0);
  }
  for (int k = 0; k < B.n; ++k) {
    B.norm[k] = 0.0;
    for (int i = 0; i < vs.q; ++i) {
      double v = 0.0;
      for (int m = 0; m < B.ncomp[k]; ++m)
        v += B.sgn[k][m] * hermite3(vs, i, B.comp[k][m][0], B.comp[k][m][1], B.comp[k][m][2]);
      B.P[k][i] = v;
      B.norm[k] += vs.w[i] * v * v;
    }
  }
  return B;
}

/* out_i = w_i sum_P P_i <A, P> / |P|^2 for a symmetric tensor A[3][3][3]. */
template <class T>
void third_order_term(const VelSet& vs, const H3Basis& B, const T A[3][3][3], T* out) {
  for (int i = 0; i < vs.q; ++i) out[i] = T(0.0);
  for (int k = 0; k < B.n; ++k) {
    T m(0.0);
    for (int r = 0; r < B.ncomp[k]; ++r) m += B.sgn[k][r] * A[B.comp[k][r][0]][B.comp[k][r][1]][B.comp[k][r][2]];
    T coef = m / B.norm[k];
    for (int i = 0; i < vs.q; ++i) out[i] += (vs.w[i] * B.P[k][i]) * coef;
  }
}

/* Third-order equilibrium (Eq. (11) with the H^(3) term of a_0^(3) = rho v v v). */
template <class T>
void equilibrium3(const VelSet& vs, const H3Basis& B, const T& rho, const T v[3], T* feq) {
  equilibrium(vs, rho, v, feq);
  T A[3][3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) A[a][b][c] = rho * v[a] * v[b] * v[c];
  T t[27];
  third_order_term(vs, B, A, t);
  for (int i = 0; i < vs.q; ++i) feq[i] += t[i];
}

/* Guo source term for population i: w_i [3(xi_i - v) + 9 (xi_i.v) xi_i].F. */
template <class T>
T guo_term(const VelSet& vs, int i, const T v[3], const double F[3]) {
  T cv = double(vs.c[i][0]) * v[0] + double(vs.c[i][1]) * v[1] + double(vs.c[i][2]) * v[2];
  double cF = vs.c[i][0] * F[0] + vs.c[i][1] * F[1] + vs.c[i][2] * F[2];
  T vF = v[0] * F[0] + v[1] * F[1] + v[2] * F[2];
  return vs.w[i] * (3.0 * (T(cF) - vF) + 9.0 * cv * cF);
}

/* Effective relaxation time of the Smagorinsky BGK model (Eqs. (3),(4),(14)):
 * the positive root of tau^2 - tau0 tau - 9 C_S^2 |Pi| / (sqrt(2) rho) = 0. */
template <class T, class C>
T tau_effective(double tau0, const C& cs, const T& pinorm, const T& rho) {
  return 0.5 * (tau0 + sqrt(tau0 * tau0 + 18.0 * std::sqrt(2.0) * cs * cs * pinorm / rho));
}

/* ------------------------------------------------------------------------ */
/* Spalding wall function (Sec. 2.2.1, Eq. (17)), smooth wall:               */
/*   y+ = g(u+) = u+ + [exp(a) - 1 - a - a^2/2 - a^3/6] / E,  a = kappa u+.   */
/* For small a the bracket is evaluated by its power series sum_{n>=4}       */
/* a^n/n!, which avoids the cancellation of the four leading terms.          */
/* ------------------------------------------------------------------------ */
double exp_tail(double a, int from) {
  /* sum_{n >= from} a^n / n!  for 0 <= a < 1/2 (from = 3 or 4) */
  double term = 1.0;
  for (int n = 1; n <= from; ++n) term *= a / n;
  double sum = 0.0;
  for (int n = from; n < from + 24; ++n) {
    sum += term;
    term *= a / (n + 1);
  }
  return sum;
}
double spalding_g(double up, double kappa, double E) {
  double k = kappa * up;
  double rem = (k >= 0.0 && k < 0.5) ? exp_tail(k, 4) : std::exp(k) - 1.0 - k - 0.5 * k * k - k * k * k / 6.0;
  return up + rem / E;
}
double spalding_dg(double up, double kappa, double E) {
  double k = kappa * up;
  double rem = (k >= 0.0 && k < 0.5) ? exp_tail(k, 3) : std::exp(k) - 1.0 - k - 0.5 * k * k;
  return 1.0 + kappa * rem / E;
}

/* Friction velocity from the law at distance y with tangential speed U:
 * root of F(ut) = g(U/ut) - y ut / nu.  F is convex and decreasing and the
 * laminar guess sqrt(nu U / y) has F >= 0, so Newton climbs monotonically. */
int solve_utau(double U, double y, double nu, double kappa, double E, double* utau, int* iters) {
  double ut = std::sqrt(nu * U / y);
  if (!(kappa * U / ut <= 700.0)) return ORC_ENEWTON;
  for (int it = 1; it <= 100; ++it) {
    double x = U / ut;
    double Fv = spalding_g(x, kappa, E) - y * ut / nu;
    double dF = -spalding_dg(x, kappa, E) * U / (ut * ut) - y / nu;
    double step = -Fv / dF;
    ut += step;
    if (std::fabs(step) <= 1e-15 * ut) {
      *utau = ut;
      if (iters) *iters = it;
      return ORC_OK;
    }
  }
  return ORC_ENEWTON;
}

/* An upper bound of the root of g(u+) = y+: the root is below y+ (g(u) >= u),
 * so exp(kappa u+) = E(y+ - u+) + 1 + k + k^2/2 + k^3/6 with k = kappa u+
 * is at most E y+ + 1 + K + K^2/2 + K^3/6 with K = kappa y+. */
double uplus_upper_bound(double yplus, double kappa, double E) {
  double K = kappa * yplus;
  double b = std::log(E * yplus + 1.0 + K + 0.5 * K * K + K * K * K / 6.0) / kappa;
  return std::fmin(yplus, b);
}

/* Inverse of the law: u+ with g(u+) = y+, Newton from a start right of the
 * root (g is convex and increasing there, so the iterates decrease). */
int solve_uplus(double yplus, double start, double kappa, double E, double* uplus) {
  double u = start;
  if (!(kappa * u <= 700.0)) return ORC_ENEWTON;
  for (int it = 1; it <= 100; ++it) {
    double step = -(spalding_g(u, kappa, E) - yplus) / spalding_dg(u, kappa, E);
    u += step;
    if (std::fabs(step) <= 1e-15 * std::fabs(u)) {
      *uplus = u;
      return ORC_OK;
    }
  }
  return ORC_ENEWTON;
}

enum Kind : uint8_t { K_SOLID = 0, K_BULK = 1, K_WALL = 2, K_LID = 3, K_INLET = 4, K_OUTLET = 5 };

/* ------------------------------------------------------------------------ */
/* The simulation state.                                                     */
/* ------------------------------------------------------------------------ */
struct SimBase {
  virtual ~SimBase() {}
  std::string err;
  virtual int step(int n) = 0;
  virtual int moments(double* rho, double* u) = 0;
  virtual int diagnostics(double* out) = 0;
  virtual int get_populations(double* f, double* df) = 0;
  virtual int set_populations(const double* f, const double* df) = 0;
  virtual int set_phi_tangent(const double* dphi) = 0;
  virtual int set_smagorinsky(const double* cs, const double* dcs) = 0;
  virtual int objective(const int planes[2], double* J, double* dJ) = 0;
  virtual int wall_info(long* cells, long* refs, double* normal, double* utau, double* G, double* tau) = 0;
  virtual int wall_velocity(double* tangent, double* utan) = 0;
  virtual int set_vortices(int n, const double* yz, const int* sign, double intensity, double sigma) = 0;
  virtual long num_wall() const = 0;
  virtual int get_post_collision(double* f) = 0;
};

template <class T>
struct Sim : SimBase {
  orc_params p;
  VelSet vs;
  H3Basis h3;
  long N = 0;
  std::vector<uint8_t> fluid, kind;
  std::vector<T> phi;
  /* per-cell Smagorinsky constant (the dynamics take C_S from the cell,
   * Sec. 2.3); empty: the scalar cs_smag everywhere */
  std::vector<T> csf;
  T cs_at(long c) const { return csf.empty() ? T(p.cs_smag) : csf[c]; }
  std::vector<T> f, fs; /* [q][N]: state f^n and post-collision f* */
  /* wall-model geometry (fixed at creation) */
  std::vector<long> wcell, wref;
  std::vector<double> wnorm, wyb, wyr;
  std::vector<long> wall_index; /* cell -> wall record, -1 if none */
  /* pre-collision velocity field [3][N] of the current step (hybrid collision only) */
  std::vector<T> uf;
  /* wall-model records of the current step (FP64 values; in tangent mode
   * they carry their derivatives too) */
  std::vector<T> wt, wutan, wG, wtau, wutau;
  /* inflow vortices of the vortex method: positions (y, z), circulations */
  std::vector<double> vy, vz, vgam;
  double vsig = 1.0;

  long idx(int x, int y, int z) const { return x + (long)p.nx * (y + (long)p.ny * z); }
  /* The equilibrium of the selected collision model (second or third order). */
  void eqm(const T& rho, const T v[3], T* feq) const {
    if (p.collision == 1) equilibrium3(vs, h3, rho, v, feq);
    else equilibrium(vs, rho, v, feq);
  }
  void coords(long c, int& x, int& y, int& z) const {
    x = int(c % p.nx);
    y = int((c / p.nx) % p.ny);
    z = int(c / ((long)p.nx * p.ny));
  }
  /* Cell at (x,y,z) + (dx,dy,dz) with periodic wrap; -1 if outside a non-periodic axis. */
  long neighbor_xyz(int x, int y, int z, int dx, int dy, int dz) const {
    int q[3] = {x + dx, y + dy, z + dz};
    const int n[3] = {p.nx, p.ny, p.nz};
    for (int a = 0; a < 3; ++a) {
      if (q[a] < 0 || q[a] >= n[a]) {
        if (!p.periodic[a]) return -1;
        q[a] = (q[a] % n[a] + n[a]) % n[a];
      }
    }
    return idx(q[0], q[1], q[2]);
  }
  long neighbor(long c, int dx, int dy, int dz) const {
    int x, y, z;
    coords(c, x, y, z);
    return neighbor_xyz(x, y, z, dx, dy, dz);
  }
  bool is_fluid(long c) const { return c >= 0 && fluid[c]; }
  /* Full-slip faces: the axes along which the move (x, y, z) + d leaves the
   * box, when every face it crosses is a full-slip face; 0 when the move
   * stays inside or crosses any other face. */
  int slip_cross(int x, int y, int z, int dx, int dy, int dz) const {
    if (!p.slip) return 0;
    const int q[3] = {x + dx, y + dy, z + dz};
    const int n[3] = {p.nx, p.ny, p.nz};
    int m = 0;
    for (int a = 0; a < 3; ++a) {
      if (p.periodic[a]) continue;
      if (q[a] < 0) {
        if (!((p.slip >> (2 * a)) & 1)) return 0;
        m |= 1 << a;
      } else if (q[a] >= n[a]) {
        if (!((p.slip >> (2 * a + 1)) & 1)) return 0;
        m |= 1 << a;
      }
    }
    return m;
  }
  int dir_index(const int c[3]) const {
    for (int i = 0; i < vs.q; ++i)
      if (vs.c[i][0] == c[0] && vs.c[i][1] == c[1] && vs.c[i][2] == c[2]) return i;
    return -1;
  }

  /* Log-law inflow profile of the urban setup: u_ref ln(1+z_c/z0)/ln(1+z_top/z0). */
  double u_in(double zc) const {
    double ztop = p.nz - 0.5;
    return p.u_ref * std::log(1.0 + zc / p.z0) / std::log(1.0 + ztop / p.z0);
  }

  /* Vortex method (Sec. 2.2.2): seed points p_i on the inflow plane with
   * signs s_i; k_i = 3/2 (|u_mean(p_i)| I)^2 and
   * Gamma_i = 4 s_i sqrt(pi / (6 ln 3 - 9 ln 2) k_i A / n), A the inlet area
   * (ny nz cells).  The inflow direction is d = +x. */
  int set_vortices(int n, const double* yz, const int* sign, double intensity, double sigma) override {
    if (!p.open_x || n < 0 || (n > 0 && (!yz || !sign)) || !(sigma > 0.0) || !std::isfinite(sigma) ||
        !(intensity >= 0.0) || !std::isfinite(intensity)) {
      err = "vortices need open x faces, n >= 0, positions and signs, sigma > 0 and intensity >= 0";
      return ORC_EINVAL;
    }
    for (int i = 0; i < n; ++i)
      if (!(yz[2 * i] >= 0.0 && yz[2 * i] <= p.ny && yz[2 * i + 1] >= 0.0 && yz[2 * i + 1] <= p.nz)) {
        err = "vortex positions must lie on the inflow plane";
        return ORC_EINVAL;
      }
    const double pi = 3.14159265358979323846;
    vy.assign(n, 0.0);
    vz.assign(n, 0.0);
    vgam.assign(n, 0.0);
    vsig = sigma;
    const double A = double(p.ny) * p.nz;
    for (int i = 0; i < n; ++i) {
      vy[i] = yz[2 * i];
      vz[i] = yz[2 * i + 1];
      const double um = std::fabs(u_in(vz[i]));
      const double k = 1.5 * (um * intensity) * (um * intensity);
      const double s = sign[i] >= 0 ? 1.0 : -1.0;
      vgam[i] = 4.0 * s * std::sqrt(pi / (6.0 * std::log(3.0) - 9.0 * std::log(2.0)) * k * A / n);
    }
    return ORC_OK;
  }
  /* u_vortex(x) = 1/(2 pi) sum_i Gamma_i ((p_i - x) x d)(1 - exp(-|x - p_i|^2 / (2 sigma^2))) / |x - p_i|^2
   * at the point (y, z) of the inflow plane; with d = +x,
   * (p - x) x d = (0, (p - x)_z, -(p - x)_y).  The exponent's sign is the
   * decaying one (the printed formula grows without bound). */
  void u_vortex(double y, double z, double u[3]) const {
    const double pi = 3.14159265358979323846;
    u[0] = u[1] = u[2] = 0.0;
    for (size_t i = 0; i < vgam.size(); ++i) {
      const double dy = vy[i] - y, dz = vz[i] - z;
      const double r2 = dy * dy + dz * dz;
      if (r2 == 0.0) continue;
      const double f = vgam[i] / (2.0 * pi) * (1.0 - std::exp(-r2 / (2.0 * vsig * vsig))) / r2;
      u[1] += f * dz;
      u[2] -= f * dy;
    }
  }

  int init(const orc_params* prm, const uint8_t* mask, const double* wall_dist, const double* porosity,
           const double* rho0, const double* u0) {
    p = *prm;
    if (!(p.q == 19 || p.q == 27) || p.nx <= 0 || p.ny <= 0 || p.nz <= 0) {
      err = "invalid lattice or size";
      return ORC_EINVAL;
    }
    if (!(p.tau0 > 0.5) || !(p.cs_smag >= 0.0)) {
      err = "tau0 must exceed 1/2 and C_S must be >= 0";
      return ORC_EINVAL;
    }
    if (p.collision != 0 && p.collision != 1) {
      err = "collision must be 0 (BGK) or 1 (recursive regularized)";
      return ORC_EINVAL;
    }
    if (!(p.fd_weight >= 0.0 && p.fd_weight <= 1.0) || (p.fd_weight > 0.0 && p.collision != 1)) {
      err = "fd_weight must be in [0, 1], and above 0 only with the recursive regularized collision";
      return ORC_EINVAL;
    }
    if (p.open_x != 0 && p.open_x != 1) {
      err = "open_x must be 0 or 1";
      return ORC_EINVAL;
    }
    if (p.open_x &&
        (p.periodic[0] || p.nx < 3 || p.fringe_len > p.nx - 2 || p.fd_weight > 0.0 || p.force[0] != 0.0 ||
         p.force[1] != 0.0 || p.force[2] != 0.0 || !(p.rho_out > 0.0) || !std::isfinite(p.rho_out) ||
         !(p.z0 > 0.0) || !std::isfinite(p.u_ref))) {
      err = "open x faces need a non-periodic x axis, nx >= 3, fringe_len <= nx - 2, no hybrid, no force, "
            "rho_out > 0 and the inflow profile (z0 > 0, finite u_ref)";
      return ORC_EINVAL;
    }
    for (int a = 0; a < 3; ++a)
      if (p.periodic[a] && ((p.slip >> (2 * a)) & 3)) {
        err = "full-slip faces need a non-periodic axis";
        return ORC_EINVAL;
      }
    if ((p.slip & ~63) || (p.open_x && (p.slip & 3)) || (p.lid && (p.slip & 32))) {
      err = "full-slip faces: six face bits, not on open x faces, not on the top face with a lid";
      return ORC_EINVAL;
    }
    vs = make_velocity_set(p.q);
    h3 = make_h3_basis(vs);
    N = (long)p.nx * p.ny * p.nz;
    fluid.assign(N, 1);
    if (mask)
      for (long c = 0; c < N; ++c) fluid[c] = mask[c] ? 1 : 0;
    phi.assign(N, T(1.0));
    if (porosity)
      for (long c = 0; c < N; ++c) phi[c] = T(porosity[c]);
    /* classify cells */
    kind.assign(N, K_SOLID);
    for (long c = 0; c < N; ++c) {
      if (!fluid[c]) continue;
      int x, y, z;
      coords(c, x, y, z);
      kind[c] = (p.lid && z == p.nz - 1) ? K_LID : K_BULK;
      if (p.open_x && kind[c] == K_BULK && x == 0) kind[c] = K_INLET;
      if (p.open_x && kind[c] == K_BULK && x == p.nx - 1) kind[c] = K_OUTLET;
    }
    wall_index.assign(N, -1);
    if (p.wall_model) {
      if (!wall_dist) {
        err = "wall model needs a wall-distance field";
        return ORC_EINVAL;
      }
      for (long b = 0; b < N; ++b) {
        if (kind[b] != K_BULK) continue;
        int s[3] = {0, 0, 0};
        bool any = false;
        int bx, by, bz;
        coords(b, bx, by, bz);
        for (int i = 1; i < vs.q; ++i) {
          long nb = neighbor(b, vs.c[i][0], vs.c[i][1], vs.c[i][2]);
          /* links through full-slip faces are not walls of the wall model */
          if (!is_fluid(nb) && !slip_cross(bx, by, bz, vs.c[i][0], vs.c[i][1], vs.c[i][2])) {
            any = true;
            for (int a = 0; a < 3; ++a) s[a] -= vs.c[i][a];
          }
        }
        if (!any || (s[0] == 0 && s[1] == 0 && s[2] == 0)) continue; /* bulk (plain bounce-back) */
        /* reference direction: argmax (xi.s)/|xi|, exact integer comparison,
         * ties to the lowest index */
        int best = -1;
        long bdot = 0, bn2 = 1;
        for (int i = 1; i < vs.q; ++i) {
          long d = vs.c[i][0] * s[0] + vs.c[i][1] * s[1] + vs.c[i][2] * s[2];
          long n2 = vs.c[i][0] * vs.c[i][0] + vs.c[i][1] * vs.c[i][1] + vs.c[i][2] * vs.c[i][2];
          bool better;
          if (best < 0) better = true;
          else if ((d > 0) != (bdot > 0) || (d == 0) != (bdot == 0)) better = (d > bdot);
          else if (d > 0) better = d * d * bn2 > bdot * bdot * n2;
          else better = d * d * bn2 < bdot * bdot * n2; /* both <= 0 */
          if (better) { best = i; bdot = d; bn2 = n2; }
        }
        long r = neighbor(b, vs.c[best][0], vs.c[best][1], vs.c[best][2]);
        if (!is_fluid(r)) r = b;
        double yb = wall_dist[b], yr = wall_dist[r];
        if (!(yb > 0.0 && std::isfinite(yb) && yr > 0.0 && std::isfinite(yr))) {
          err = "wall distance must be positive and finite at wall cells and their references";
          return ORC_EINVAL;
        }
        double sn = std::sqrt(double(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]));
        wall_index[b] = (long)wcell.size();
        wcell.push_back(b);
        wref.push_back(r);
        for (int a = 0; a < 3; ++a) wnorm.push_back(s[a] / sn);
        wyb.push_back(yb);
        wyr.push_back(yr);
        kind[b] = K_WALL;
      }
    }
    long nw = (long)wcell.size();
    wt.assign(3 * nw, T(0.0));
    wutan.assign(nw, T(0.0));
    wG.assign(nw, T(0.0));
    wtau.assign(nw, T(p.tau0));
    wutau.assign(nw, T(0.0));
    /* initial populations: equilibrium of the initial density and velocity */
    f.assign((size_t)vs.q * N, T(0.0));
    fs.assign((size_t)vs.q * N, T(0.0));
    for (long c = 0; c < N; ++c) {
      if (!fluid[c]) continue;
      T r = rho0 ? T(rho0[c]) : T(1.0);
      T v[3];
      for (int a = 0; a < 3; ++a) v[a] = u0 ? T(u0[(size_t)a * N + c]) : T(0.0);
      T feq[27];
      eqm(r, v, feq);
      for (int i = 0; i < vs.q; ++i) f[(size_t)i * N + c] = feq[i];
    }
    return ORC_OK;
  }

  void local_moments(long c, T& rho, T j[3]) const {
    rho = T(0.0);
    j[0] = j[1] = j[2] = T(0.0);
    for (int i = 0; i < vs.q; ++i) {
      T fi = f[(size_t)i * N + c];
      rho += fi;
      for (int a = 0; a < 3; ++a) j[a] += double(vs.c[i][a]) * fi;
    }
  }

  /* A root found by Newton in double precision, as a value of type T: in
   * tangent mode its derivative follows from the implicit function theorem,
   * d root = -(dF/dp) dp / (dF/droot) for the residual F(root, p) = 0. */
  static T root_of(double v, const T& param, double dF_dparam, double dF_droot) {
    if constexpr (std::is_same<T, Dual>::value) return Dual(v, -dF_dparam * der(param) / dF_droot);
    else return T(v);
  }

  /* Wall prepass: u_tau, modeled tangential speed and strain from f^n.  In
   * tangent mode the records carry their derivatives: through the reference
   * cell's velocity, the tangent direction, and the two Newton solves
   * (implicit derivatives of their roots). */
  int wall_prepass() {
    const double nu = (p.tau0 - 0.5) / 3.0;
    int status = ORC_OK;
    long nw = (long)wcell.size();
    for (long k = 0; k < nw; ++k) {
      long r = wref[k];
      T rho;
      T j[3];
      local_moments(r, rho, j);
      T u[3];
      for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * p.force[a]) / rho;
      const double* n = &wnorm[3 * k];
      T un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
      T ut[3] = {u[0] - un * n[0], u[1] - un * n[1], u[2] - un * n[2]};
      T U = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
      const double Uv = val(U);
      if (!(Uv > 1e-300)) {
        wt[3 * k] = wt[3 * k + 1] = wt[3 * k + 2] = T(0.0);
        wutan[k] = T(0.0);
        wG[k] = T(0.0);
        wutau[k] = T(0.0);
        wtau[k] = T(3.0 * nu + 0.5);
        continue;
      }
      double utv = 0.0;
      int rc = solve_utau(Uv, wyr[k], nu, p.kappa, p.E, &utv, nullptr);
      if (rc != ORC_OK) { status = rc; continue; }
      /* F(u_tau; U) = g(U/u_tau) - y_r u_tau / nu */
      const double gpr = spalding_dg(Uv / utv, p.kappa, p.E);
      T utau = root_of(utv, U, gpr / utv, -gpr * Uv / (utv * utv) - wyr[k] / nu);
      T uplus_b;
      if (r == wcell[k]) {
        uplus_b = U / utau;
      } else {
        double yplus_b = wyb[k] * utv / nu;
        double start = uplus_upper_bound(yplus_b, p.kappa, p.E);
        if (wyr[k] >= wyb[k]) start = std::fmin(start, Uv / utv);
        double upv;
        rc = solve_uplus(yplus_b, start, p.kappa, p.E, &upv);
        if (rc != ORC_OK) { status = rc; continue; }
        /* G(u+; u_tau) = g(u+) - y_b u_tau / nu */
        uplus_b = root_of(upv, utau, -wyb[k] / nu, spalding_dg(upv, p.kappa, p.E));
      }
      for (int a = 0; a < 3; ++a) wt[3 * k + a] = ut[a] / U;
      wutan[k] = utau * uplus_b;
      const T csb = cs_at(wcell[k]);
      T cs2 = csb * csb;
      T G = 2.0 * utau * utau / (nu + sqrt(nu * nu + 4.0 * cs2 * utau * utau));
      wG[k] = G;
      wutau[k] = utau;
      wtau[k] = 3.0 * (nu + cs2 * G) + 0.5;
    }
    if (status != ORC_OK) err = "wall-function Newton solve failed (no convergence or exp range)";
    return status;
  }

  /* Velocity field of the current state (Guo velocity, fluid cells). */
  void velocity_field() {
    uf.assign((size_t)3 * N, T(0.0));
    for (long c = 0; c < N; ++c) {
      if (!fluid[c]) continue;
      T r, j[3];
      local_moments(c, r, j);
      for (int a = 0; a < 3; ++a) uf[(size_t)a * N + c] = (j[a] + 0.5 * p.force[a]) / r;
    }
  }
  /* Strain rate S_ab = (d_a u_b + d_b u_a)/2 at cell c by central differences
   * of the velocity field; one-sided where one neighbour along the axis is not
   * fluid, zero where neither is. */
  void strain_fd(long c, T S[3][3]) const {
    T D[3][3];
    for (int a = 0; a < 3; ++a) {
      int e[3] = {0, 0, 0};
      e[a] = 1;
      long xp = neighbor(c, e[0], e[1], e[2]), xm = neighbor(c, -e[0], -e[1], -e[2]);
      bool fp = is_fluid(xp), fm = is_fluid(xm);
      for (int b = 0; b < 3; ++b) {
        T uc = uf[(size_t)b * N + c];
        if (fp && fm) D[a][b] = 0.5 * (uf[(size_t)b * N + xp] - uf[(size_t)b * N + xm]);
        else if (fp) D[a][b] = uf[(size_t)b * N + xp] - uc;
        else if (fm) D[a][b] = uc - uf[(size_t)b * N + xm];
        else D[a][b] = T(0.0);
      }
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) S[a][b] = 0.5 * (D[a][b] + D[b][a]);
  }

  /* Bulk cell (sigma = 1): homogenized Smagorinsky collision with Guo
   * forcing; BGK (collision 0) keeps all of f - f^eq, the recursive
   * regularized model (collision 1) keeps its Hermite reconstruction. */
  bool collide_bulk(long c, T* fo) const {
    T fi[27];
    for (int i = 0; i < vs.q; ++i) fi[i] = f[(size_t)i * N + c];
    return collide_populations(c, fi, fo);
  }
  /* The same collision of the given pre-collision populations of cell c. */
  bool collide_populations(long c, const T* fi, T* fo) const {
    T rho(0.0), j[3] = {T(0.0), T(0.0), T(0.0)};
    for (int i = 0; i < vs.q; ++i) {
      rho += fi[i];
      for (int a = 0; a < 3; ++a) j[a] += double(vs.c[i][a]) * fi[i];
    }
    T u[3];
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * p.force[a]) / rho;
    T feq[27];
    eqm(rho, u, feq);
    T Pi[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Pi[a][b] = T(0.0);
    for (int i = 0; i < vs.q; ++i) {
      T fneq = fi[i] - feq[i];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Pi[a][b] += double(vs.c[i][a] * vs.c[i][b]) * fneq;
    }
    T pi2(0.0);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) pi2 += Pi[a][b] * Pi[a][b];
    T tau = tau_effective(p.tau0, cs_at(c), sqrt(pi2), rho);
    T uh[3];
    for (int a = 0; a < 3; ++a) uh[a] = phi[c] * u[a];
    T feqh[27];
    eqm(rho, uh, feqh);
    if (p.collision == 1) {
      /* f^(1) from its Hermite coefficients (Eqs. (8), (9), n = 0..3):
       * a^(0) = sum f^(1) = 0; a^(1) = sum xi f^(1) (with the Guo velocity
       * this is -F/2); a^(2) = Pi; and by the recursion
       * a^(3)_abc = u_a Pi_bc + u_b Pi_ac + u_c Pi_ab */
      T a1[3] = {T(0.0), T(0.0), T(0.0)};
      for (int i = 0; i < vs.q; ++i)
        for (int a = 0; a < 3; ++a) a1[a] += double(vs.c[i][a]) * (fi[i] - feq[i]);
      T A[3][3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          for (int g = 0; g < 3; ++g) A[a][b][g] = u[a] * Pi[b][g] + u[b] * Pi[a][g] + u[g] * Pi[a][b];
      T t3[27];
      third_order_term(vs, h3, A, t3);
      /* hybrid (Eq. (7)): the second-order part blends Pi with the stress of
       * the finite-difference strain, -2 rho c_s^2 tau S^FD (f^(1,FD) of
       * Eq. (10)); the third-order part keeps the factor sigma */
      const double sig = 1.0 - p.fd_weight;
      T Ph[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Ph[a][b] = Pi[a][b];
      if (p.fd_weight > 0.0) {
        T S[3][3];
        strain_fd(c, S);
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) Ph[a][b] = sig * Pi[a][b] - p.fd_weight * (2.0 / 3.0) * rho * tau * S[a][b];
        for (int i = 0; i < vs.q; ++i) t3[i] = sig * t3[i];
      }
      T trPi = Ph[0][0] + Ph[1][1] + Ph[2][2];
      for (int i = 0; i < vs.q; ++i) {
        T cPc(0.0);
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) cPc += double(vs.c[i][a] * vs.c[i][b]) * Ph[a][b];
        T ca1 = double(vs.c[i][0]) * a1[0] + double(vs.c[i][1]) * a1[1] + double(vs.c[i][2]) * a1[2];
        /* w_i H^(1)_i . a^(1) / c_s^2 = 3 w_i xi.a1;
         * w_i H^(2)_i : Pi / (2 c_s^4) = 9/2 w_i (xi.Pi.xi - c_s^2 tr Pi) */
        T f1 = 3.0 * vs.w[i] * ca1 + 4.5 * vs.w[i] * (cPc - trPi / 3.0) + t3[i];
        fo[i] = feqh[i] + (1.0 - 1.0 / tau) * f1 + (1.0 - 0.5 / tau) * guo_term(vs, i, u, p.force);
      }
    } else {
      for (int i = 0; i < vs.q; ++i)
        fo[i] = feqh[i] + (1.0 - 1.0 / tau) * (fi[i] - feq[i]) +
                (1.0 - 0.5 / tau) * guo_term(vs, i, u, p.force);
    }
    return std::isfinite(val(rho)) && val(rho) > 0.0;
  }

  /* Open-face cell (inlet or outlet): its pre-collision populations rebuilt
   * by the regularized local condition (reading in the header).  n is the
   * outward normal, -x at the inlet and +x at the outlet; the populations
   * with xi.n < 0 enter through the face and are unknown. */
  void open_reconstruct(long c, T* fr) const {
    int x, y, z;
    coords(c, x, y, z);
    const bool inlet = kind[c] == K_INLET;
    const int nx_out = inlet ? -1 : 1; /* x component of the outward normal */
    T fi[27];
    for (int i = 0; i < vs.q; ++i) fi[i] = f[(size_t)i * N + c];
    /* mass and normal momentum of the known populations: sum over xi.n = 0
     * and over the populations leaving through the face (xi.n > 0) */
    T s_par(0.0), s_out(0.0);
    for (int i = 0; i < vs.q; ++i) {
      const int cn = vs.c[i][0] * nx_out;
      if (cn == 0) s_par += fi[i];
      else if (cn > 0) s_out += fi[i];
    }
    /* rho = s_par + s_out + s_in and rho u.n = s_out - s_in give
     * rho (1 + u.n) = s_par + 2 s_out */
    T rho, u[3];
    if (inlet) {
      double uv[3];
      u_vortex(y + 0.5, z + 0.5, uv);
      u[0] = T(u_in(z + 0.5));
      u[1] = T(uv[1]);
      u[2] = T(uv[2]);
      const T un = double(nx_out) * u[0];
      rho = (s_par + 2.0 * s_out) / (1.0 + un);
    } else {
      rho = T(p.rho_out);
      const T un = (s_par + 2.0 * s_out) / rho - 1.0;
      u[0] = double(nx_out) * un;
      u[1] = u[2] = T(0.0);
    }
    T feq[27];
    eqm(rho, u, feq);
    if (!inlet) {
      /* the outlet holds the equilibrium at (rho_out, u): a non-equilibrium
       * rebuilt there from the arriving populations feeds the over-relaxed
       * (tau near 1/2) non-equilibrium back through the face and grows */
      for (int i = 0; i < vs.q; ++i) fr[i] = feq[i];
      return;
    }
    /* inlet non-equilibrium: known populations as they are, an unknown one
     * takes that of its opposite direction */
    T fneq[27];
    for (int i = 0; i < vs.q; ++i) {
      const bool unknown = vs.c[i][0] * nx_out < 0;
      fneq[i] = unknown ? fi[vs.opp[i]] - feq[vs.opp[i]] : fi[i] - feq[i];
    }
    T Pi[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        Pi[a][b] = T(0.0);
        for (int i = 0; i < vs.q; ++i) Pi[a][b] += double(vs.c[i][a] * vs.c[i][b]) * fneq[i];
      }
    const T trPi = Pi[0][0] + Pi[1][1] + Pi[2][2];
    for (int i = 0; i < vs.q; ++i) {
      T cPc(0.0);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) cPc += double(vs.c[i][a] * vs.c[i][b]) * Pi[a][b];
      /* w_i H^(2)_i : Pi / (2 c_s^4) = 9/2 w_i (xi.Pi.xi - c_s^2 tr Pi) */
      fr[i] = feq[i] + 4.5 * vs.w[i] * (cPc - trPi / 3.0);
    }
  }

  /* Wall cell (sigma = 0): equilibrium at the modeled velocity plus the
   * non-equilibrium built from the wall-law strain S = (G/2)(t n^T + n t^T). */
  bool collide_wall(long c, long k, T* fo) const {
    T rho(0.0), j[3] = {T(0.0), T(0.0), T(0.0)};
    for (int i = 0; i < vs.q; ++i) {
      T fi = f[(size_t)i * N + c];
      rho += fi;
      for (int a = 0; a < 3; ++a) j[a] += double(vs.c[i][a]) * fi;
    }
    const double* n = &wnorm[3 * k];
    const T* t = &wt[3 * k];
    T u[3];
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * p.force[a]) / rho;
    T un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
    T uw[3];
    for (int a = 0; a < 3; ++a) uw[a] = wutan[k] * t[a] + un * n[a];
    T tau = wtau[k], G = wG[k];
    T feq[27];
    eqm(rho, uw, feq);
    /* with the hybrid collision, the full finite-difference strain whose
     * wall-normal shear (the tangential part s of S n, in every tangential
     * direction) is replaced by the wall law's, G/2 along t:
     * S' = S - (s n^T + n s^T) + (G/2)(t n^T + n t^T), s = S n - (n.S.n) n */
    T S[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) S[a][b] = T(0.0);
    if (p.fd_weight > 0.0) {
      strain_fd(c, S);
      T Sn[3], nSn(0.0);
      for (int a = 0; a < 3; ++a) {
        Sn[a] = S[a][0] * n[0] + S[a][1] * n[1] + S[a][2] * n[2];
        nSn += n[a] * Sn[a];
      }
      T sv[3];
      for (int a = 0; a < 3; ++a) sv[a] = Sn[a] - nSn * n[a];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          S[a][b] = S[a][b] - (sv[a] * n[b] + n[a] * sv[b]) + 0.5 * G * (t[a] * n[b] + n[a] * t[b]);
    } else {
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S[a][b] = 0.5 * G * (t[a] * n[b] + n[a] * t[b]);
    }
    T trS = S[0][0] + S[1][1] + S[2][2];
    for (int i = 0; i < vs.q; ++i) {
      T cSc(0.0);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) cSc += double(vs.c[i][a] * vs.c[i][b]) * S[a][b];
      /* f^(1,FD)_i = -(w_i rho tau / c_s^2) H^(2)_i : S */
      T ffd = -3.0 * vs.w[i] * rho * tau * (cSc - trS / 3.0);
      fo[i] = feq[i] + (1.0 - 1.0 / tau) * ffd + (1.0 - 0.5 / tau) * guo_term(vs, i, uw, p.force);
    }
    return std::isfinite(val(rho)) && val(rho) > 0.0;
  }

  int step_once() {
    if (p.fd_weight > 0.0) velocity_field();
    if (p.wall_model && !wcell.empty()) {
      int rc = wall_prepass();
      if (rc != ORC_OK) return rc;
    }
    int bad = 0;
    const int fstart = p.nx - p.fringe_len;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int z = 0; z < p.nz; ++z)
      for (int y = 0; y < p.ny; ++y)
        for (int x = 0; x < p.nx; ++x) {
          long c = idx(x, y, z);
          if (!fluid[c]) continue;
          T fo[27];
          if (kind[c] == K_LID) {
            T v[3] = {T(u_in(p.nz - 0.5)), T(0.0), T(0.0)};
            eqm(T(1.0), v, fo);
          } else if (kind[c] == K_WALL) {
            if (!collide_wall(c, wall_index[c], fo)) bad = 1;
          } else if (kind[c] == K_INLET || kind[c] == K_OUTLET) {
            T fr[27];
            open_reconstruct(c, fr);
            if (!collide_populations(c, fr, fo)) bad = 1;
          } else {
            if (!collide_bulk(c, fo)) bad = 1;
          }
          if (p.fringe_len > 0 && x >= fstart && kind[c] != K_OUTLET) {
            double s = double(x - fstart + 1) / p.fringe_len;
            double lam = s * s * (3.0 - 2.0 * s);
            T v[3] = {T(u_in(z + 0.5)), T(0.0), T(0.0)};
            T fin[27];
            eqm(T(1.0), v, fin);
            for (int i = 0; i < vs.q; ++i) fo[i] = (1.0 - lam) * fo[i] + lam * fin[i];
          }
          for (int i = 0; i < vs.q; ++i) fs[(size_t)i * N + c] = fo[i];
        }
    /* pull streaming with halfway bounce-back; across full-slip faces the
     * population is reflected specularly: f_i(x) = f*_j(x - c_i with the
     * crossed components set to zero), c_j = c_i with those components
     * negated, when that cell is fluid (else bounce-back) */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p.nz; ++z)
      for (int y = 0; y < p.ny; ++y)
        for (int x = 0; x < p.nx; ++x) {
          long c = idx(x, y, z);
          if (!fluid[c]) continue;
          for (int i = 0; i < vs.q; ++i) {
            long src = neighbor_xyz(x, y, z, -vs.c[i][0], -vs.c[i][1], -vs.c[i][2]);
            if (is_fluid(src)) {
              f[(size_t)i * N + c] = fs[(size_t)i * N + src];
              continue;
            }
            const int m = slip_cross(x, y, z, -vs.c[i][0], -vs.c[i][1], -vs.c[i][2]);
            long rsrc = -1;
            int j = -1;
            if (m) {
              int d[3], cj[3];
              for (int a = 0; a < 3; ++a) {
                const bool crossed = (m >> a) & 1;
                d[a] = crossed ? 0 : -vs.c[i][a];
                cj[a] = crossed ? -vs.c[i][a] : vs.c[i][a];
              }
              rsrc = neighbor_xyz(x, y, z, d[0], d[1], d[2]);
              j = dir_index(cj);
            }
            f[(size_t)i * N + c] = is_fluid(rsrc) ? fs[(size_t)j * N + rsrc] : fs[(size_t)vs.opp[i] * N + c];
          }
        }
    if (bad) {
      err = "non-finite or non-positive density";
      return ORC_ENONFINITE;
    }
    return ORC_OK;
  }

  int step(int n) override {
    for (int s = 0; s < n; ++s) {
      int rc = step_once();
      if (rc != ORC_OK) return rc;
    }
    return ORC_OK;
  }

  int moments(double* rho, double* u) override {
    for (long c = 0; c < N; ++c) {
      if (!fluid[c]) {
        if (rho) rho[c] = 0.0;
        if (u) u[c] = u[N + c] = u[2 * N + c] = 0.0;
        continue;
      }
      T r, j[3];
      local_moments(c, r, j);
      if (rho) rho[c] = val(r);
      if (u)
        for (int a = 0; a < 3; ++a) u[(size_t)a * N + c] = val((j[a] + 0.5 * p.force[a]) / r);
    }
    return ORC_OK;
  }

  int diagnostics(double* out) override {
    double M = 0, P[3] = {0, 0, 0};
    for (long c = 0; c < N; ++c) {
      if (!fluid[c]) continue;
      T r, j[3];
      local_moments(c, r, j);
      M += val(r);
      for (int a = 0; a < 3; ++a) P[a] += val(j[a]);
    }
    out[0] = M;
    out[1] = P[0];
    out[2] = P[1];
    out[3] = P[2];
    return ORC_OK;
  }

  int get_populations(double* fo, double* dfo) override {
    for (size_t k = 0; k < f.size(); ++k) {
      if (fo) fo[k] = val(f[k]);
      if (dfo) dfo[k] = der(f[k]);
    }
    return ORC_OK;
  }

  int set_populations(const double* fi, const double* dfi) override;
  int set_phi_tangent(const double* dphi) override;
  /* per-cell Smagorinsky constants (and, in tangent mode, their direction) */
  int set_smagorinsky(const double* cs, const double* dcs) override {
    if (!cs) {
      csf.clear();
      return ORC_OK;
    }
    for (long c = 0; c < N; ++c)
      if (!(cs[c] >= 0.0) || !std::isfinite(cs[c])) {
        err = "Smagorinsky constants must be finite and >= 0";
        return ORC_EINVAL;
      }
    csf.assign(N, T(0.0));
    for (long c = 0; c < N; ++c) {
      if constexpr (std::is_same<T, Dual>::value) csf[c] = Dual(cs[c], dcs ? dcs[c] : 0.0);
      else csf[c] = T(cs[c]);
    }
    return ORC_OK;
  }

  /* Terminal objective of the porosity-gradient study: pressure drop between
   * two x-planes plus mean kinetic energy (both over fluid cells). */
  int objective(const int planes[2], double* J, double* dJ) override {
    T s0(0.0), s1(0.0), ke(0.0);
    long n0 = 0, n1 = 0, nf = 0;
    for (long c = 0; c < N; ++c) {
      if (!fluid[c]) continue;
      int x, y, z;
      coords(c, x, y, z);
      T r, j[3];
      local_moments(c, r, j);
      T m[3];
      for (int a = 0; a < 3; ++a) m[a] = j[a] + 0.5 * p.force[a];
      ke += 0.5 * (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / r;
      ++nf;
      if (x == planes[0]) { s0 += r; ++n0; }
      if (x == planes[1]) { s1 += r; ++n1; }
    }
    if (n0 == 0 || n1 == 0 || nf == 0) {
      err = "objective planes hold no fluid cell";
      return ORC_EINVAL;
    }
    T Jv = (1.0 / 3.0) * (s0 / double(n0) - s1 / double(n1)) + ke / double(nf);
    if (J) *J = val(Jv);
    if (dJ) *dJ = der(Jv);
    return ORC_OK;
  }

  long num_wall() const override { return (long)wcell.size(); }
  /* post-collision populations f* of the last step, [q][N] */
  int get_post_collision(double* fo) override {
    for (size_t k = 0; k < fs.size(); ++k) fo[k] = val(fs[k]);
    return ORC_OK;
  }
  int wall_info(long* cells, long* refs, double* normal, double* utau, double* G, double* tau) override {
    long nw = (long)wcell.size();
    for (long k = 0; k < nw; ++k) {
      if (cells) cells[k] = wcell[k];
      if (refs) refs[k] = wref[k];
      if (normal)
        for (int a = 0; a < 3; ++a) normal[3 * k + a] = wnorm[3 * k + a];
      if (utau) utau[k] = val(wutau[k]);
      if (G) G[k] = val(wG[k]);
      if (tau) tau[k] = val(wtau[k]);
    }
    return ORC_OK;
  }
  /* tangent t and modeled tangential speed u_tau u+_b of every wall record */
  int wall_velocity(double* tangent, double* utan) override {
    long nw = (long)wcell.size();
    for (long k = 0; k < nw; ++k) {
      if (tangent)
        for (int a = 0; a < 3; ++a) tangent[3 * k + a] = val(wt[3 * k + a]);
      if (utan) utan[k] = val(wutan[k]);
    }
    return ORC_OK;
  }
};

template <>
int Sim<double>::set_populations(const double* fi, const double*) {
  for (size_t k = 0; k < f.size(); ++k) f[k] = fi[k];
  return ORC_OK;
}
template <>
int Sim<Dual>::set_populations(const double* fi, const double* dfi) {
  for (size_t k = 0; k < f.size(); ++k) f[k] = Dual(fi[k], dfi ? dfi[k] : 0.0);
  return ORC_OK;
}
template <>
int Sim<double>::set_phi_tangent(const double*) {
  err = "tangent seeds need a dual-number oracle";
  return ORC_EINVAL;
}
template <>
int Sim<Dual>::set_phi_tangent(const double* dphi) {
  for (long c = 0; c < N; ++c) phi[c].d = dphi ? dphi[c] : 0.0;
  return ORC_OK;
}

thread_local std::string g_create_error;

}  // namespace

extern "C" {

/* Creates a simulation.  tangent = 0: plain FP64; tangent = 1: dual numbers
 * (directional derivatives of everything, the wall model included). */
void* orc_create(const orc_params* p, const uint8_t* mask, const double* wall_dist, const double* porosity,
                 const double* rho0, const double* u0, int tangent) {
  g_create_error.clear();
  if (!p) {
    g_create_error = "null parameters";
    return nullptr;
  }
  SimBase* s;
  int rc;
  if (tangent) {
    auto* t = new Sim<Dual>();
    rc = t->init(p, mask, wall_dist, porosity, rho0, u0);
    s = t;
  } else {
    auto* t = new Sim<double>();
    rc = t->init(p, mask, wall_dist, porosity, rho0, u0);
    s = t;
  }
  if (rc != ORC_OK) {
    g_create_error = s->err;
    delete s;
    return nullptr;
  }
  return s;
}
const char* orc_create_error(void) { return g_create_error.c_str(); }
const char* orc_last_error(void* h) { return h ? static_cast<SimBase*>(h)->err.c_str() : "null handle"; }
void orc_free(void* h) { delete static_cast<SimBase*>(h); }
int orc_step(void* h, int n) { return static_cast<SimBase*>(h)->step(n); }
int orc_moments(void* h, double* rho, double* u) { return static_cast<SimBase*>(h)->moments(rho, u); }
int orc_diagnostics(void* h, double* out) { return static_cast<SimBase*>(h)->diagnostics(out); }
int orc_get_populations(void* h, double* f, double* df) {
  return static_cast<SimBase*>(h)->get_populations(f, df);
}
int orc_set_populations(void* h, const double* f, const double* df) {
  return static_cast<SimBase*>(h)->set_populations(f, df);
}
int orc_set_phi_tangent(void* h, const double* dphi) { return static_cast<SimBase*>(h)->set_phi_tangent(dphi); }
int orc_set_smagorinsky(void* h, const double* cs, const double* dcs) {
  return static_cast<SimBase*>(h)->set_smagorinsky(cs, dcs);
}
int orc_objective(void* h, const int* planes, double* J, double* dJ) {
  return static_cast<SimBase*>(h)->objective(planes, J, dJ);
}
int orc_get_post_collision(void* h, double* f) { return static_cast<SimBase*>(h)->get_post_collision(f); }
long orc_num_wall(void* h) { return static_cast<SimBase*>(h)->num_wall(); }
int orc_set_vortices(void* h, int n, const double* yz, const int* sign, double intensity, double sigma) {
  return static_cast<SimBase*>(h)->set_vortices(n, yz, sign, intensity, sigma);
}
int orc_wall_info(void* h, long* cells, long* refs, double* normal, double* utau, double* G, double* tau) {
  return static_cast<SimBase*>(h)->wall_info(cells, refs, normal, utau, G, tau);
}
int orc_wall_velocity(void* h, double* tangent, double* utan) {
  return static_cast<SimBase*>(h)->wall_velocity(tangent, utan);
}

/* Pure helpers exposed for the pin tests. */
int orc_velocity_set(int q, int* c, double* w, int* opp) {
  if (q != 19 && q != 27) return ORC_EINVAL;
  VelSet v = make_velocity_set(q);
  for (int i = 0; i < q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = v.c[i][a];
    w[i] = v.w[i];
    opp[i] = v.opp[i];
  }
  return ORC_OK;
}
void orc_equilibrium(int q, double rho, const double* u, double* feq) {
  VelSet v = make_velocity_set(q);
  double uu[3] = {u[0], u[1], u[2]};
  equilibrium(v, rho, uu, feq);
}
void orc_equilibrium3(int q, double rho, const double* u, double* feq) {
  VelSet v = make_velocity_set(q);
  H3Basis B = make_h3_basis(v);
  double uu[3] = {u[0], u[1], u[2]};
  equilibrium3(v, B, rho, uu, feq);
}
double orc_tau_eff(double tau0, double cs, double pinorm, double rho) {
  return tau_effective(tau0, cs, pinorm, rho);
}
/* One bulk-cell collision of populations fin (FP64), porosity phi;
 * collision 0 = BGK, 1 = recursive regularized. */
void orc_collide_bulk2(int q, int collision, double tau0, double cs, const double* force, double phi,
                       const double* fin, double* fout) {
  Sim<double> s;
  s.p = orc_params{};
  s.p.q = q;
  s.p.collision = collision;
  s.p.fd_weight = 0.0;
  s.p.tau0 = tau0;
  s.p.cs_smag = cs;
  for (int a = 0; a < 3; ++a) s.p.force[a] = force[a];
  s.vs = make_velocity_set(q);
  s.h3 = make_h3_basis(s.vs);
  s.N = 1;
  s.f.assign(fin, fin + q);
  s.phi.assign(1, phi);
  s.collide_bulk(0, fout);
}
void orc_collide_bulk(int q, double tau0, double cs, const double* force, double phi, const double* fin,
                      double* fout) {
  orc_collide_bulk2(q, 0, tau0, cs, force, phi, fin, fout);
}
/* One wall-cell reconstruction collision for given wall records. */
void orc_collide_wall(int q, double tau0, double cs, const double* force, const double* fin, const double* normal,
                      const double* tangent, double utan, double G, double tau, double* fout) {
  Sim<double> s;
  s.p = orc_params{};
  s.p.q = q;
  s.p.tau0 = tau0;
  s.p.cs_smag = cs;
  for (int a = 0; a < 3; ++a) s.p.force[a] = force[a];
  s.vs = make_velocity_set(q);
  s.N = 1;
  s.f.assign(fin, fin + q);
  s.wnorm.assign(normal, normal + 3);
  s.wt.assign(tangent, tangent + 3);
  s.wutan.assign(1, utan);
  s.wG.assign(1, G);
  s.wtau.assign(1, tau);
  s.collide_wall(0, 0, fout);
}
double orc_spalding_yplus(double uplus, double kappa, double E) { return spalding_g(uplus, kappa, E); }
int orc_spalding_uplus(double yplus, double kappa, double E, double* uplus) {
  return solve_uplus(yplus, uplus_upper_bound(yplus, kappa, E), kappa, E, uplus);
}
int orc_solve_utau(double U, double y, double nu, double kappa, double E, double* utau, int* iters) {
  return solve_utau(U, y, nu, kappa, E, utau, iters);
}
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
/* Sets the number of OpenMP threads of later steps (n >= 1). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

}  /* extern "C" */
