// Host preprocessing of the voxel geometry: cell flags, the wall-cell list
// with normals and reference cells (wall model of Sec. 2.2.1), and the voxel
// wall distance.  Runs once in lbm_init; multithreaded over z-slabs.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "internal.h"
#include "lattice.h"

namespace lbmk {

namespace {

// Runs body(z0, z1) over [0, nz) split into contiguous slabs, one per thread.
template <typename F>
void parallel_slabs(int nz, F body) {
  unsigned nt = std::max(1u, std::min(std::thread::hardware_concurrency(), 64u));
  nt = std::min<unsigned>(nt, (unsigned)nz);
  if (nt <= 1) {
    body(0, nz);
    return;
  }
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) {
    const int z0 = (int)((long long)nz * t / nt), z1 = (int)((long long)nz * (t + 1) / nt);
    th.emplace_back([=]() { body(z0, z1); });
  }
  for (auto &x : th) x.join();
}

struct Box {
  int n[3];
  int per[3];
  int slip;  // full-slip face bits
  // whether the move (x,y,z) + d leaves the box through full-slip faces only
  bool slip_move(int x, int y, int z, int dx, int dy, int dz) const {
    const int q[3] = {x + dx, y + dy, z + dz};
    bool any = false;
    for (int a = 0; a < 3; ++a) {
      if (per[a]) continue;
      if (q[a] < 0) {
        if (!((slip >> (2 * a)) & 1)) return false;
        any = true;
      } else if (q[a] >= n[a]) {
        if (!((slip >> (2 * a + 1)) & 1)) return false;
        any = true;
      }
    }
    return any;
  }
  // neighbour of (x,y,z) + d with wrap; -1 when it leaves a non-periodic axis
  long long nb(int x, int y, int z, int dx, int dy, int dz) const {
    int q[3] = {x + dx, y + dy, z + dz};
    for (int a = 0; a < 3; ++a) {
      if (q[a] < 0 || q[a] >= n[a]) {
        if (!per[a]) return -1;
        q[a] = ((q[a] % n[a]) + n[a]) % n[a];
      }
    }
    return q[0] + (long long)n[0] * (q[1] + (long long)n[1] * q[2]);
  }
};

Box box_of(const lbm_params &p) {
  Box b;
  b.n[0] = p.nx;
  b.n[1] = p.ny;
  b.n[2] = p.nz;
  for (int a = 0; a < 3; ++a) b.per[a] = p.periodic[a] ? 1 : 0;
  b.slip = p.slip;
  return b;
}

inline bool fluid_at(const uint8_t *mask, long long c) { return c >= 0 && (mask == nullptr || mask[c] != 0); }

// Solid-link sum s = sum over links i with a non-fluid neighbour at +c_i of
// (-c_i), leaving out links through full-slip faces (not walls of the wall
// model); returns whether there is any such solid link, and in *slip whether
// there is a link through full-slip faces.
template <int Q>
bool solid_links(const Box &b, const uint8_t *mask, int x, int y, int z, int s[3], bool *slip) {
  bool any = false;
  *slip = false;
  s[0] = s[1] = s[2] = 0;
  for (int i = 1; i < Q; ++i) {
    const long long nbc = b.nb(x, y, z, Lat<Q>::c(i, 0), Lat<Q>::c(i, 1), Lat<Q>::c(i, 2));
    if (!fluid_at(mask, nbc)) {
      if (b.slip && b.slip_move(x, y, z, Lat<Q>::c(i, 0), Lat<Q>::c(i, 1), Lat<Q>::c(i, 2))) {
        *slip = true;
        continue;
      }
      any = true;
      for (int a = 0; a < 3; ++a) s[a] -= Lat<Q>::c(i, a);
    }
  }
  return any;
}

// Lattice direction with the largest cosine to s (exact integer comparison of
// (c.s)/|c|; ties to the lowest index).
template <int Q>
int best_direction(const int s[3]) {
  int best = -1;
  long long bd = 0, bn = 1;
  for (int i = 1; i < Q; ++i) {
    const long long d = (long long)Lat<Q>::c(i, 0) * s[0] + (long long)Lat<Q>::c(i, 1) * s[1] +
                        (long long)Lat<Q>::c(i, 2) * s[2];
    const long long n2 = Lat<Q>::n2(i);
    bool better;
    if (best < 0) {
      better = true;
    } else if ((d > 0) != (bd > 0) || (d == 0) != (bd == 0)) {
      better = d > bd;  // different signs (or one zero): compare the signs
    } else if (d > 0) {
      better = d * d * bn > bd * bd * n2;
    } else {
      better = d * d * bn < bd * bd * n2;
    }
    if (better) {
      best = i;
      bd = d;
      bn = n2;
    }
  }
  return best;
}

template <int Q>
int build(const lbm_params &p, const uint8_t *mask, Geometry &g, std::string &msg, bool count_only,
          long long *count) {
  const Box b = box_of(p);
  const long long N = (long long)p.nx * p.ny * p.nz;
  if (!count_only) g.flags.assign((size_t)N, 0);
  const int nz = p.nz;
  std::vector<std::vector<int>> wc(nz), wr(nz);
  std::vector<std::vector<double>> wn(nz);
  std::vector<char> any_solid(nz, 0), any_lid(nz, 0), any_open(nz, 0);
  parallel_slabs(nz, [&](int z0, int z1) {
    for (int z = z0; z < z1; ++z)
      for (int y = 0; y < p.ny; ++y)
        for (int x = 0; x < p.nx; ++x) {
          const long long c = x + (long long)p.nx * (y + (long long)p.ny * z);
          if (!fluid_at(mask, c)) continue;
          uint8_t fl = FL_FLUID;
          int s[3];
          bool slip_link = false;
          const bool solid = solid_links<Q>(b, mask, x, y, z, s, &slip_link);
          // links through full-slip faces also need the link-aware slot map
          const bool near = solid || slip_link;
          if (near) {
            fl |= FL_NEAR;
            any_solid[z] = 1;
          }
          const bool lid = p.lid && z == p.nz - 1;
          if (lid) {
            fl |= FL_LID;
            any_lid[z] = 1;
          }
          // open x faces: inlet / outlet cells (a lid cell stays a lid cell)
          const bool open = p.open_x && !lid && (x == 0 || x == p.nx - 1);
          if (open) {
            fl |= x == 0 ? FL_INLET : FL_OUTLET;
            any_open[z] = 1;
          }
          if (p.wall_model && solid && !lid && !open && (s[0] || s[1] || s[2])) {
            fl |= FL_WALL;
            const int k = best_direction<Q>(s);
            long long r = b.nb(x, y, z, Lat<Q>::c(k, 0), Lat<Q>::c(k, 1), Lat<Q>::c(k, 2));
            if (!fluid_at(mask, r)) r = c;
            wc[z].push_back((int)c);
            wr[z].push_back((int)r);
            const double sn = std::sqrt((double)(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]));
            for (int a = 0; a < 3; ++a) wn[z].push_back(s[a] / sn);
          }
          if (!count_only) g.flags[(size_t)c] = fl;
        }
  });
  long long total = 0;
  for (int z = 0; z < nz; ++z) total += (long long)wc[z].size();
  if (count) *count = total;
  if (count_only) return LBM_OK;
  g.wcell.clear();
  g.wref.clear();
  g.wnorm.clear();
  g.wcell.reserve((size_t)total);
  g.wref.reserve((size_t)total);
  g.wnorm.reserve(3 * (size_t)total);
  g.has_solid = false;
  g.has_lid = false;
  g.has_open = false;
  for (int z = 0; z < nz; ++z) {
    g.wcell.insert(g.wcell.end(), wc[z].begin(), wc[z].end());
    g.wref.insert(g.wref.end(), wr[z].begin(), wr[z].end());
    g.wnorm.insert(g.wnorm.end(), wn[z].begin(), wn[z].end());
    g.has_solid = g.has_solid || any_solid[z];
    g.has_lid = g.has_lid || any_lid[z];
    g.has_open = g.has_open || any_open[z];
  }
  (void)msg;
  return LBM_OK;
}

}  // namespace

int build_geometry(const lbm_params &p, const uint8_t *mask, Geometry &g, std::string &msg) {
  return p.lattice == 19 ? build<19>(p, mask, g, msg, false, nullptr) : build<27>(p, mask, g, msg, false, nullptr);
}

long long count_wall_cells(const lbm_params &p, const uint8_t *mask) {
  if (!p.wall_model) return 0;
  Geometry g;
  std::string msg;
  long long n = 0;
  if (p.lattice == 19) build<19>(p, mask, g, msg, true, &n);
  else build<27>(p, mask, g, msg, true, &n);
  return n;
}

// Distance from the centre of cell c to the nearest solid unit cube whose
// centre lies within two cells along every axis (outside a non-periodic
// axis counts as solid, except beyond a full-slip face, where the geometry
// continues as its mirror image); +inf when there is none.
double voxel_distance(const lbm_params &p, const uint8_t *mask, long long c) {
  const Box b = box_of(p);
  const int x = (int)(c % p.nx);
  const int y = (int)((c / p.nx) % p.ny);
  const int z = (int)(c / ((long long)p.nx * p.ny));
  double best = INFINITY;
  for (int dz = -2; dz <= 2; ++dz)
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        int q[3] = {x + dx, y + dy, z + dz};
        for (int a = 0; a < 3; ++a) {
          if (b.per[a]) continue;
          if (q[a] < 0 && ((b.slip >> (2 * a)) & 1)) q[a] = -1 - q[a];
          else if (q[a] >= b.n[a] && ((b.slip >> (2 * a + 1)) & 1)) q[a] = 2 * b.n[a] - 1 - q[a];
        }
        const long long nbc = b.nb(q[0], q[1], q[2], 0, 0, 0);
        if (fluid_at(mask, nbc)) continue;
        const double gx = std::max(std::abs(dx) - 0.5, 0.0), gy = std::max(std::abs(dy) - 0.5, 0.0),
                     gz = std::max(std::abs(dz) - 0.5, 0.0);
        best = std::min(best, std::sqrt(gx * gx + gy * gy + gz * gz));
      }
  return best;
}

}  // namespace lbmk
