// Host geometry: voxelisation, wall links, wall distances q and flag words.
#include "geometry.hpp"

#include <algorithm>
#include <cmath>
#include <thread>

#include "lattice.hpp"

namespace lbm {
namespace {

inline int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Run body(z) for z in [0, nz) on a few host threads (slabs are independent).
template <class F>
void for_each_z(int nz, F body) {
  unsigned hw = std::thread::hardware_concurrency();
  int nt = (int)std::min<unsigned>(hw ? hw : 1, 16);
  if (nz < 8 || nt <= 1) {
    for (int z = 0; z < nz; ++z) body(z);
    return;
  }
  nt = std::min(nt, nz);
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([=]() {
      for (int z = t; z < nz; z += nt) body(z);
    });
  for (auto& th : pool) th.join();
}

// Node p is solid iff |p - c'|^2 < r^2 for a sphere image c' = c + o*N,
// o in {-1,0,1}^3 (radius below the box edge, centre inside the box).
void voxelise(const lbm_sphere* sp, int ns, int nx, int ny, int nz, uint8_t* mask) {
  for_each_z(nz, [&](int z) {
    for (int s = 0; s < ns; ++s) {
      const double r = sp[s].r, r2 = r * r;
      for (int oz = -1; oz <= 1; ++oz) {
        const double cz = sp[s].cz + oz * nz;
        const double dz = z - cz;
        if (std::fabs(dz) >= r) continue;
        for (int oy = -1; oy <= 1; ++oy) {
          const double cy = sp[s].cy + oy * ny;
          const int y0 = std::max(0, (int)std::floor(cy - r)), y1 = std::min(ny - 1, (int)std::ceil(cy + r));
          for (int ox = -1; ox <= 1; ++ox) {
            const double cx = sp[s].cx + ox * nx;
            const int x0 = std::max(0, (int)std::floor(cx - r)), x1 = std::min(nx - 1, (int)std::ceil(cx + r));
            for (int y = y0; y <= y1; ++y) {
              const double dy = y - cy;
              uint8_t* row = mask + (int64_t)nx * (y + (int64_t)ny * z);
              for (int x = x0; x <= x1; ++x) {
                const double dx = x - cx;
                if (dx * dx + dy * dy + dz * dz < r2) row[x] = 1;
              }
            }
          }
        }
      }
    }
  });
}

// Wall distance of the link from fluid node (x,y,z) along e_j: the smallest
// t in [0,1] at which x + t e_j enters a sphere image.  With h = e.d,
// a = |e|^2, c0 = |d|^2 - r^2 the entry root (-h - sqrt(h^2 - a c0))/a is
// evaluated as c0 / (-h + sqrt(.)) when h < 0 to avoid cancellation.
double link_distance(const lbm_sphere* sp, int ns, int nx, int ny, int nz, int x, int y, int z,
                     int j) {
  const double ex = kLat.ex[j], ey = kLat.ey[j], ez = kLat.ez[j];
  const double a = ex * ex + ey * ey + ez * ez;
  double best = 2.0;
  for (int s = 0; s < ns; ++s) {
    const double r = sp[s].r;
    for (int oz = -1; oz <= 1; ++oz) {
      const double dz = z - (sp[s].cz + oz * nz);
      if (std::fabs(dz) > r + 1.0) continue;
      for (int oy = -1; oy <= 1; ++oy) {
        const double dy = y - (sp[s].cy + oy * ny);
        if (std::fabs(dy) > r + 1.0) continue;
        for (int ox = -1; ox <= 1; ++ox) {
          const double dx = x - (sp[s].cx + ox * nx);
          if (std::fabs(dx) > r + 1.0) continue;
          const double h = ex * dx + ey * dy + ez * dz;
          const double c0 = dx * dx + dy * dy + dz * dz - r * r;
          const double disc = h * h - a * c0;
          if (disc < 0.0) continue;
          const double sq = std::sqrt(disc);
          const double t = h < 0.0 ? c0 / (sq - h) : (-h - sq) / a;
          if (t >= 0.0 && t <= 1.0 && t < best) best = t;
        }
      }
    }
  }
  return best <= 1.0 ? best : 0.5;
}

}  // namespace

bool build_geometry(const uint8_t* mask_in, const lbm_sphere* spheres, int ns, int nx, int ny,
                    int nz, Geometry& g, std::string& err) {
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.nz_cell = nz;
  g.ncell = (int64_t)nx * ny * nz;
  g.mask.assign(g.ncell, 0);
  if (mask_in) {
    for (int64_t c = 0; c < g.ncell; ++c) g.mask[c] = mask_in[c] ? 1 : 0;
  } else {
    voxelise(spheres, ns, nx, ny, nz, g.mask.data());
  }
  g.n_fluid = 0;
  for (int64_t c = 0; c < g.ncell; ++c) g.n_fluid += g.mask[c] == 0;
  if (g.n_fluid == 0) {
    err = "geometry has no fluid cell";
    return false;
  }

  // Flags and links, per z slab, then concatenated in cell order.
  g.flags.assign(g.ncell, 0);
  std::vector<std::vector<int64_t>> cells(nz);
  std::vector<std::vector<int32_t>> dirs(nz);
  std::vector<std::vector<double>> qs(nz);
  std::vector<std::vector<uint8_t>> fbs(nz);
  const uint8_t* m = g.mask.data();
  for_each_z(nz, [&](int z) {
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t c = x + (int64_t)nx * (y + (int64_t)ny * z);
        if (m[c]) {
          // bit k: the fluid node c + e_k pulls direction k from this cell,
          // so the cell's slot in plane k holds that link's coefficient
          uint32_t f = kSolid;
          for (int k = 1; k < kQ; ++k) {
            const int xn = wrap1(x + kLat.ex[k], nx), yn = wrap1(y + kLat.ey[k], ny),
                      zn = wrap1(z + kLat.ez[k], nz);
            if (!m[xn + (int64_t)nx * (yn + (int64_t)ny * zn)]) f |= 1u << k;
          }
          g.flags[c] = f;
          continue;
        }
        uint32_t f = 0;
        for (int j = 1; j < kQ; ++j) {
          const int xs = wrap1(x + kLat.ex[j], nx), ys = wrap1(y + kLat.ey[j], ny),
                    zs = wrap1(z + kLat.ez[j], nz);
          if (!m[xs + (int64_t)nx * (ys + (int64_t)ny * zs)]) continue;
          // link (c, j): the pull of direction k = opp(j) finds a solid source
          f |= 1u << kLat.opp[j];
          const int xb = wrap1(x - kLat.ex[j], nx), yb = wrap1(y - kLat.ey[j], ny),
                    zb = wrap1(z - kLat.ez[j], nz);
          cells[z].push_back(c);
          dirs[z].push_back(j);
          qs[z].push_back(mask_in ? 0.5 : link_distance(spheres, ns, nx, ny, nz, x, y, z, j));
          fbs[z].push_back(m[xb + (int64_t)nx * (yb + (int64_t)ny * zb)] ? 1 : 0);
        }
        g.flags[c] = f;
      }
  });
  size_t total = 0;
  for (int z = 0; z < nz; ++z) total += cells[z].size();
  g.link_cell.clear();
  g.link_dir.clear();
  g.link_q.clear();
  g.link_fallback.clear();
  g.link_cell.reserve(total);
  g.link_dir.reserve(total);
  g.link_q.reserve(total);
  g.link_fallback.reserve(total);
  g.n_fallback = 0;
  for (int z = 0; z < nz; ++z) {
    g.link_cell.insert(g.link_cell.end(), cells[z].begin(), cells[z].end());
    g.link_dir.insert(g.link_dir.end(), dirs[z].begin(), dirs[z].end());
    g.link_q.insert(g.link_q.end(), qs[z].begin(), qs[z].end());
    g.link_fallback.insert(g.link_fallback.end(), fbs[z].begin(), fbs[z].end());
    for (uint8_t b : fbs[z]) g.n_fallback += b;
  }
  return true;
}

void append_cell(Geometry& g, const Geometry& c) {
  const int64_t off = g.ncell;
  if (g.ncell == 0) {
    g.nx = c.nx;
    g.ny = c.ny;
    g.nz = 0;
    g.nz_cell = c.nz;
  }
  g.nz += c.nz;
  g.ncell += c.ncell;
  g.n_fluid += c.n_fluid;
  g.n_fallback += c.n_fallback;
  g.mask.insert(g.mask.end(), c.mask.begin(), c.mask.end());
  g.flags.insert(g.flags.end(), c.flags.begin(), c.flags.end());
  for (int64_t cell : c.link_cell) g.link_cell.push_back(cell + off);
  g.link_dir.insert(g.link_dir.end(), c.link_dir.begin(), c.link_dir.end());
  g.link_q.insert(g.link_q.end(), c.link_q.begin(), c.link_q.end());
  g.link_fallback.insert(g.link_fallback.end(), c.link_fallback.begin(), c.link_fallback.end());
}

}  // namespace lbm
