// Velocity sets, storage conversions and the per-lane neighbour geometry of
// the AA in-place streaming scheme, for the gfx950 kernels.
//
// D3Q19 is the stencil of the paper (Sec. 2.2, lattice figure); D3Q27 adds
// the eight corner directions.  Order: rest, nine "positive" directions
// (D3Q27: then four corners with +x), then the negatives in the same order,
// so the opposite of i is i +- (q-1)/2.  Weights: D3Q19 1/3, 1/18, 1/36;
// D3Q27 8/27, 2/27, 1/54, 1/216 (rest, axis, edge, corner).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace lbmk {

template <int Q>
struct Lat {
  static_assert(Q == 19 || Q == 27, "D3Q19 or D3Q27");
  static constexpr int H = (Q - 1) / 2;  // number of "positive" directions
  __host__ __device__ static constexpr int c(int i, int a) {
    constexpr int pos[13][3] = {{1, 0, 0}, {0, 1, 0},  {0, 0, 1},  {1, 1, 0},  {1, -1, 0},
                                {1, 0, 1}, {1, 0, -1}, {0, 1, 1},  {0, 1, -1}, {1, 1, 1},
                                {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
    return i == 0 ? 0 : (i <= H ? pos[i - 1][a] : -pos[i - 1 - H][a]);
  }
  __host__ __device__ static constexpr int opp(int i) { return i == 0 ? 0 : (i <= H ? i + H : i - H); }
  __host__ __device__ static constexpr int n2(int i) {
    return c(i, 0) * c(i, 0) + c(i, 1) * c(i, 1) + c(i, 2) * c(i, 2);
  }
  __host__ __device__ static constexpr double w(int i) {
    return Q == 19 ? (n2(i) == 0 ? 1.0 / 3.0 : n2(i) == 1 ? 1.0 / 18.0 : 1.0 / 36.0)
                   : (n2(i) == 0 ? 8.0 / 27.0 : n2(i) == 1 ? 2.0 / 27.0 : n2(i) == 2 ? 1.0 / 54.0 : 1.0 / 216.0);
  }
};

// ---------------------------------------------------------------------------
// Third-order Hermite terms of the recursive regularized collision (Sec. 2.2,
// Eqs. (8), (9), (11)).  H3_abc(c_i) = c_a c_b c_c - c_s^2 (c_a d_bc + c_b d_ac
// + c_c d_ab).  A symmetric third-order tensor is held by its seven
// components that can matter on these lattices, in the order
//   0 xxy, 1 xxz, 2 xyy, 3 yyz, 4 xzz, 5 yzz, 6 xyz
// (xxx-type components vanish: c^3 = c).  The basis polynomials a lattice
// carries, orthogonal in the weighted lattice sum sum_i w_i P_k P_l:
//   D3Q27: the seven components themselves;
//   D3Q19: xyz vanishes and the pairs (xxy, yzz), (xzz, xyy), (yyz, xxz)
//          alias, so their sums and differences.
// A tensor A enters the populations as w_i sum_k P_k(c_i) <A, P_k> / |P_k|^2
// with the lattice norms |P_k|^2 = sum_i w_i P_k(c_i)^2.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int t3_axis(int comp, int r) {
  constexpr int T[7][3] = {{0, 0, 1}, {0, 0, 2}, {0, 1, 1}, {1, 1, 2}, {0, 2, 2}, {1, 2, 2}, {0, 1, 2}};
  return T[comp][r];
}
template <int Q>
__host__ __device__ constexpr double h3(int i, int comp) {
  const int a = t3_axis(comp, 0), b = t3_axis(comp, 1), c = t3_axis(comp, 2);
  const double ca = Lat<Q>::c(i, a), cb = Lat<Q>::c(i, b), cc = Lat<Q>::c(i, c);
  return ca * cb * cc - (ca * (b == c) + cb * (a == c) + cc * (a == b)) / 3.0;
}
template <int Q>
struct H3Basis {
  static constexpr int n = Q == 27 ? 7 : 6;
  // first and second component of basis polynomial k, and the sign of the
  // second (0: a single component)
  __host__ __device__ static constexpr int c0(int k) {
    constexpr int A[6] = {0, 0, 4, 4, 3, 3};
    return Q == 27 ? k : A[k];
  }
  __host__ __device__ static constexpr int c1(int k) {
    constexpr int B[6] = {5, 5, 2, 2, 1, 1};
    return Q == 27 ? 0 : B[k];
  }
  __host__ __device__ static constexpr double sgn(int k) { return Q == 27 ? 0.0 : (k % 2 == 0 ? 1.0 : -1.0); }
  __host__ __device__ static constexpr double P(int k, int i) {
    return h3<Q>(i, c0(k)) + (sgn(k) != 0.0 ? sgn(k) * h3<Q>(i, c1(k)) : 0.0);
  }
};
template <int Q>
struct H3Norms {
  double v[7];
};
template <int Q>
__host__ __device__ constexpr H3Norms<Q> h3_norms() {
  H3Norms<Q> r{};
  for (int k = 0; k < H3Basis<Q>::n; ++k) {
    double s = 0.0;
    for (int i = 0; i < Q; ++i) s += Lat<Q>::w(i) * H3Basis<Q>::P(k, i) * H3Basis<Q>::P(k, i);
    r.v[k] = s;
  }
  return r;
}
__host__ __device__ constexpr bool near_eq(double a, double b) { return a - b < 1e-15 && b - a < 1e-15; }
// D3Q27: 2 c_s^6 for the xxy type, c_s^6 for xyz; D3Q19: 2 c_s^6 for the sums,
// 6 c_s^6 for the differences (the continuous norm of each sum and difference
// would be 4 c_s^6).
static_assert(near_eq(h3_norms<27>().v[0], 2.0 / 27.0) && near_eq(h3_norms<27>().v[6], 1.0 / 27.0), "D3Q27 norms");
static_assert(near_eq(h3_norms<19>().v[0], 2.0 / 27.0) && near_eq(h3_norms<19>().v[1], 6.0 / 27.0), "D3Q19 norms");

// s += c * v for a lattice component c in {-1, 0, 1} known at compile time
// after unrolling (no multiplication, no 0*v).
template <typename R>
__device__ __forceinline__ void acc(R &s, int c, R v) {
  if (c > 0) s += v;
  else if (c < 0) s -= v;
}
template <typename R>
__device__ __forceinline__ R dot3(int cx, int cy, int cz, R x, R y, R z) {
  R s = R(0);
  acc(s, cx, x);
  acc(s, cy, y);
  acc(s, cz, z);
  return s;
}

// Smagorinsky coefficient of the cell: 18 sqrt(2) C_S^2 multiplies |Pi|/rho
// under the root of tau_eff (Sec. 2.3).  C_S comes from the cell's field when
// the context holds one (the dynamics read it per cell), else the scalar.
constexpr double SMAG_COEF = 25.455844122715710878430397035774;  // 18 sqrt(2)
template <typename R>
__device__ __forceinline__ R smag_of(const KArgs &k, int cell) {
  if (k.csf) {
    const R c = static_cast<const R *>(k.csf)[cell];
    return R(SMAG_COEF) * c * c;
  }
  return R(k.smag);
}
// C_S of the cell in FP64 (gradients with respect to C_S).
template <typename R>
__device__ __forceinline__ double cs_of(const KArgs &k, int cell) {
  return k.csf ? (double)static_cast<const R *>(k.csf)[cell] : k.cs;
}
// C_S^2 of the cell in FP64 (wall records).
template <typename R>
__device__ __forceinline__ double cs2_of(const KArgs &k, int cell) {
  if (k.csf) {
    const double c = (double)static_cast<const R *>(k.csf)[cell];
    return c * c;
  }
  return k.cs2;
}

// Stored value type -> compute type.
template <typename S>
struct Store;
template <>
struct Store<double> {
  using R = double;
  static __device__ __forceinline__ R ld(const double *p) { return *p; }
  static __device__ __forceinline__ void st(double *p, R v) { *p = v; }
};
template <>
struct Store<float> {
  using R = float;
  static __device__ __forceinline__ R ld(const float *p) { return *p; }
  static __device__ __forceinline__ void st(float *p, R v) { *p = v; }
};
template <>
struct Store<_Float16> {
  using R = float;
  static __device__ __forceinline__ R ld(const _Float16 *p) { return (float)*p; }
  static __device__ __forceinline__ void st(_Float16 *p, R v) { *p = (_Float16)v; }  // round to nearest even
};

// Neighbour geometry of one cell: offsets (in cells) to the -1 / +1 neighbour
// along each axis with periodic wrap, and which moves leave the domain
// through a non-periodic face (those links count as solid).  These and the
// slot functions below also compile for the host, where lbm_slot_map
// evaluates the same map for inspection.
struct Nb {
  int cell;
  int d[3][2];
  unsigned out;   // bit 2a: -1 along axis a leaves the domain; bit 2a+1: +1 does
  unsigned slip;  // the bits of out whose face is a full-slip face
};

__host__ __device__ __forceinline__ Nb make_nb(int x, int y, int z, const KArgs &k) {
  Nb n;
  const int sy = k.nx, sz = k.nx * k.ny;
  n.cell = x + sy * y + sz * z;
  n.d[0][0] = (x == 0) ? (k.nx - 1) : -1;
  n.d[0][1] = (x == k.nx - 1) ? -(k.nx - 1) : 1;
  n.d[1][0] = (y == 0) ? (k.ny - 1) * sy : -sy;
  n.d[1][1] = (y == k.ny - 1) ? -(k.ny - 1) * sy : sy;
  n.d[2][0] = (z == 0) ? (k.nz - 1) * sz : -sz;
  n.d[2][1] = (z == k.nz - 1) ? -(k.nz - 1) * sz : sz;
  unsigned o = 0;
  if (!k.per[0]) o |= (x == 0 ? 1u : 0u) | (x == k.nx - 1 ? 2u : 0u);
  if (!k.per[1]) o |= (y == 0 ? 4u : 0u) | (y == k.ny - 1 ? 8u : 0u);
  if (!k.per[2]) o |= (z == 0 ? 16u : 0u) | (z == k.nz - 1 ? 32u : 0u);
  n.out = o;
  n.slip = o & (unsigned)k.slip;
  return n;
}

__host__ __device__ __forceinline__ void cell_xyz(int c, const KArgs &k, int &x, int &y, int &z) {
  x = c % k.nx;
  int t = c / k.nx;
  y = t % k.ny;
  z = t / k.ny;
}

// Offset of the cell at + sgn * c_i.
template <int Q>
__host__ __device__ __forceinline__ int nb_off(const Nb &n, int i, int sgn) {
  int o = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int c = sgn * Lat<Q>::c(i, a);
    if (c < 0) o += n.d[a][0];
    else if (c > 0) o += n.d[a][1];
  }
  return o;
}
template <int Q>
__host__ __device__ __forceinline__ bool nb_out(const Nb &n, int i, int sgn) {
  bool r = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int c = sgn * Lat<Q>::c(i, a);
    if (c < 0) r = r || ((n.out >> (2 * a)) & 1u);
    else if (c > 0) r = r || ((n.out >> (2 * a + 1)) & 1u);
  }
  return r;
}

// Face bits (2a: low face of axis a, 2a+1: high face) crossed by the move
// + sgn * c_i, and the axes they belong to.
template <int Q>
__host__ __device__ __forceinline__ unsigned cross_faces(const Nb &n, int i, int sgn) {
  unsigned r = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int c = sgn * Lat<Q>::c(i, a);
    if (c < 0) r |= n.out & (1u << (2 * a));
    else if (c > 0) r |= n.out & (1u << (2 * a + 1));
  }
  return r;
}
__host__ __device__ __forceinline__ unsigned face_axes(unsigned faces) {
  return ((faces | (faces >> 1)) & 1u) | (((faces >> 2) | (faces >> 3)) & 1u) << 1 |
         (((faces >> 4) | (faces >> 5)) & 1u) << 2;
}
// Specular reflection at full-slip faces: the offset of the move + sgn * c_i
// with its components along `axes` set to zero, and the direction of c_i
// with those components negated.
template <int Q>
__host__ __device__ __forceinline__ int reflect_off(const Nb &n, int i, int sgn, unsigned axes) {
  int o = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if ((axes >> a) & 1u) continue;
    const int c = sgn * Lat<Q>::c(i, a);
    if (c < 0) o += n.d[a][0];
    else if (c > 0) o += n.d[a][1];
  }
  return o;
}
template <int Q>
__host__ __device__ constexpr int dir_of(int cx, int cy, int cz) {
  for (int j = 0; j < Q; ++j)
    if (Lat<Q>::c(j, 0) == cx && Lat<Q>::c(j, 1) == cy && Lat<Q>::c(j, 2) == cz) return j;
  return -1;
}
template <int Q>
__host__ __device__ constexpr int reflect_dir_const(int i, unsigned axes) {
  return dir_of<Q>((axes & 1u) ? -Lat<Q>::c(i, 0) : Lat<Q>::c(i, 0), (axes & 2u) ? -Lat<Q>::c(i, 1) : Lat<Q>::c(i, 1),
                   (axes & 4u) ? -Lat<Q>::c(i, 2) : Lat<Q>::c(i, 2));
}
// i is a compile-time constant after unrolling; axes (1..7) is not.
template <int Q>
__host__ __device__ __forceinline__ int reflect_dir(int i, unsigned axes) {
  int j = i;
#pragma unroll
  for (unsigned m = 1; m < 8; ++m)
    if (axes == m) j = reflect_dir_const<Q>(i, m);
  return j;
}

// Link mask of a cell.  Bit i (0..31): the upstream cell (cell - c_i) is
// solid or outside, so f_i arrives by halfway bounce-back.  Bit 32 + i: the
// upstream move leaves the box through full-slip faces only and the
// specularly reflected source (that move with the crossed components set to
// zero) is fluid, so f_i arrives by specular reflection.
// SLIP = false (no full-slip faces: every link leaving the box is solid)
// compiles without any of the reflection code; kernels take SLIP = true only
// for domains with full-slip faces.
using LinkMask = uint64_t;
template <int Q, bool SLIP = false>
__host__ __device__ __forceinline__ LinkMask solid_mask(const Nb &n, const uint8_t *__restrict__ flags) {
  if constexpr (!SLIP) {
    unsigned m = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const bool s = nb_out<Q>(n, i, -1) || !(flags[n.cell + nb_off<Q>(n, i, -1)] & FL_FLUID);
      m |= (s ? 1u : 0u) << i;
    }
    return (LinkMask)m;
  } else {
    LinkMask m = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const unsigned cf = cross_faces<Q>(n, i, -1);
      bool s, sl = false;
      if (cf == 0u) {
        s = !(flags[n.cell + nb_off<Q>(n, i, -1)] & FL_FLUID);
      } else if ((cf & ~n.slip) == 0u) {
        sl = (flags[n.cell + reflect_off<Q>(n, i, -1, face_axes(cf))] & FL_FLUID) != 0;
        s = !sl;
      } else {
        s = true;
      }
      m |= (LinkMask)(s ? 1u : 0u) << i;
      m |= (LinkMask)(sl ? 1u : 0u) << (32 + i);
    }
    return m;
  }
}

// AA pattern (in-place, one buffer A[i][cell]).
// Even parity: the state f_i(x) sits at A[i][x]; the post-collision f*_i(x)
//   is written to A[opp i][x].
// Odd parity: the state f_i(x) is A[opp i][x - c_i] if that cell is fluid,
//   else A[i][x] (halfway bounce-back); f*_i(x) goes to A[i][x + c_i] if that
//   cell is fluid, else to A[opp i][x].
// Across full-slip faces (specular reflection, c_j = c_i with the crossed
//   components negated): at odd parity f_i(x) is A[opp j][x - c_i with the
//   crossed components zeroed], where the even step left f*_j of that cell,
//   and f*_i(x) goes to A[j][x + c_i with the crossed components zeroed],
//   where the next even step reads f_j of that cell.
// Each cell reads and writes the same set of slots, and the sets of two cells
// are disjoint, so every cell can be updated concurrently in place (the
// reflected slots of a face row form the same kind of bijection as the
// bounce-back slots they replace).
template <int Q, bool ODD, bool SLIP = false>
__host__ __device__ __forceinline__ size_t read_slot(const Nb &n, LinkMask sm, int i, size_t N) {
  if (!ODD) return (size_t)i * N + (size_t)n.cell;
  if ((sm >> i) & 1u) return (size_t)i * N + (size_t)n.cell;
  if (SLIP && ((sm >> (32 + i)) & 1u)) {
    const unsigned ax = face_axes(cross_faces<Q>(n, i, -1));
    return (size_t)Lat<Q>::opp(reflect_dir<Q>(i, ax)) * N + (size_t)(n.cell + reflect_off<Q>(n, i, -1, ax));
  }
  return (size_t)Lat<Q>::opp(i) * N + (size_t)(n.cell + nb_off<Q>(n, i, -1));
}
template <int Q, bool ODD, bool SLIP = false>
__host__ __device__ __forceinline__ size_t write_slot(const Nb &n, LinkMask sm, int i, size_t N) {
  if (!ODD) return (size_t)Lat<Q>::opp(i) * N + (size_t)n.cell;
  if ((sm >> Lat<Q>::opp(i)) & 1u) return (size_t)Lat<Q>::opp(i) * N + (size_t)n.cell;
  if (SLIP && ((sm >> (32 + Lat<Q>::opp(i))) & 1u)) {
    const unsigned ax = face_axes(cross_faces<Q>(n, i, +1));
    return (size_t)reflect_dir<Q>(i, ax) * N + (size_t)(n.cell + reflect_off<Q>(n, i, +1, ax));
  }
  return (size_t)i * N + (size_t)(n.cell + nb_off<Q>(n, i, +1));
}

// Plain-path slot addressing (cells with no solid link): direction of the
// slot and its element index within that direction's array.  The element
// index is a 32-bit offset from a per-direction base that is uniform across
// the wavefront, which keeps the address arithmetic in 32 bits.
template <int Q, bool ODD>
__host__ __device__ __forceinline__ int plain_read(const Nb &n, int i, int &dir) {
  dir = ODD ? Lat<Q>::opp(i) : i;
  return ODD ? n.cell + nb_off<Q>(n, i, -1) : n.cell;
}
template <int Q, bool ODD>
__host__ __device__ __forceinline__ int plain_write(const Nb &n, int i, int &dir) {
  dir = ODD ? i : Lat<Q>::opp(i);
  return ODD ? n.cell + nb_off<Q>(n, i, +1) : n.cell;
}
// Element idx of direction array dir; requires N * sizeof(S) <= 2^32 (checked
// when the context is created).
template <typename S>
__device__ __forceinline__ S *slot_at(S *pop, int dir, size_t N, int idx) {
  return reinterpret_cast<S *>(reinterpret_cast<char *>(pop + (size_t)dir * N) +
                               (size_t)((uint32_t)idx * (uint32_t)sizeof(S)));
}

// Third-order Hermite coefficients K_k = <A, P_k> / |P_k|^2 of a tensor given
// by its components A[0..6] (xxy, xxz, xyy, yyz, xzz, yzz, xyz).
template <int Q, typename R>
__device__ __forceinline__ void third_coefs(const R A[7], R K[7]) {
  constexpr H3Norms<Q> nrm = h3_norms<Q>();
#pragma unroll
  for (int k = 0; k < H3Basis<Q>::n; ++k) {
    R m = A[H3Basis<Q>::c0(k)];
    if (H3Basis<Q>::sgn(k) > 0.0) m += A[H3Basis<Q>::c1(k)];
    if (H3Basis<Q>::sgn(k) < 0.0) m -= A[H3Basis<Q>::c1(k)];
    K[k] = m * R(1.0 / nrm.v[k]);
  }
}
// sum_k P_k(c_i) K_k (the caller multiplies by w_i).
template <int Q, typename R>
__device__ __forceinline__ R third_term(int i, const R K[7]) {
  R v = R(0);
#pragma unroll
  for (int k = 0; k < H3Basis<Q>::n; ++k) {
    const double p = H3Basis<Q>::P(k, i);
    if (p != 0.0) v += R(p) * K[k];
  }
  return v;
}
// Components of rho v v v.
template <typename R>
__device__ __forceinline__ void cube_tensor(R rho, R vx, R vy, R vz, R A[7]) {
  const R rx = rho * vx, ry = rho * vy;
  A[0] = rx * vx * vy;
  A[1] = rx * vx * vz;
  A[2] = rx * vy * vy;
  A[3] = ry * vy * vz;
  A[4] = rx * vz * vz;
  A[5] = ry * vz * vz;
  A[6] = rx * vy * vz;
}

// XCD-aware block order: hardware hands block b to XCD b % 8; give each XCD
// a contiguous run of tiles so that neighbouring tiles share its L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb) {
  const unsigned q = nb >> 3, r = nb & 7u, x = b & 7u, s = b >> 3;
  return x * q + (x < r ? x : r) + s;
}


// Strain rate S = (D + D^T)/2 of the step's velocity field at cell n, with
// D_ab = d_a u_b by central differences; one-sided where one neighbour along
// the axis is solid or outside a non-periodic axis, zero where both are
// (hybrid collision, Sec. 2.2, Eq. (10)).  S[0..5] = xx, yy, zz, xy, xz, yz.
// The velocity field of the hybrid is one vector per cell, (u_x, u_y, u_z,
// rho) at a fluid cell and 0 elsewhere (rho > 0 marks the fluid cells): a
// neighbour's velocity and whether it is fluid come in one vector load.
template <typename R>
struct alignas(4 * sizeof(R)) V4 {
  R x, y, z, w;
};

template <typename R>
__device__ __forceinline__ void fd_strain(const Nb &n, const KArgs &k, R S[6]) {
  const V4<R> *v = static_cast<const V4<R> *>(k.vel);
  const V4<R> c = v[n.cell];
  R D[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const V4<R> zero = {R(0), R(0), R(0), R(0)};
    const V4<R> P = ((n.out >> (2 * a + 1)) & 1u) ? zero : v[n.cell + n.d[a][1]];
    const V4<R> M = ((n.out >> (2 * a)) & 1u) ? zero : v[n.cell + n.d[a][0]];
    const bool fp = P.w > R(0), fm = M.w > R(0);
    const R up[3] = {P.x, P.y, P.z}, um[3] = {M.x, M.y, M.z}, uc[3] = {c.x, c.y, c.z};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (fp && fm) D[a][b] = R(0.5) * (up[b] - um[b]);
      else if (fp) D[a][b] = up[b] - uc[b];
      else if (fm) D[a][b] = uc[b] - um[b];
      else D[a][b] = R(0);
    }
  }
  S[0] = D[0][0];
  S[1] = D[1][1];
  S[2] = D[2][2];
  S[3] = R(0.5) * (D[0][1] + D[1][0]);
  S[4] = R(0.5) * (D[0][2] + D[2][0]);
  S[5] = R(0.5) * (D[1][2] + D[2][1]);
}

}  // namespace lbmk
