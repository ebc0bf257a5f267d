// Drives the host geometry of the GPU library (voxelisation, wall links,
// wall distances, flag words, batch stacking) on random sphere packs and
// masks, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
// (test infrastructure).  Checks that the flag words agree with the mask.
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "geometry.hpp"
#include "lattice.hpp"

using namespace lbm;

static bool consistent(const Geometry& g) {
  const int64_t n = g.ncell;
  if ((int64_t)g.mask.size() != n || (int64_t)g.flags.size() != n) return false;
  for (int64_t c = 0; c < n; ++c) {
    const bool solid = (g.flags[c] & kSolid) != 0;
    if (solid != (g.mask[c] != 0)) return false;
  }
  for (size_t i = 0; i < g.link_cell.size(); ++i) {
    const int64_t c = g.link_cell[i];
    if (c < 0 || c >= n || g.mask[c]) return false;
    const double q = g.link_q[i];
    if (!(q >= 0.0 && q <= 1.0)) return false;
    if (!(g.flags[c] & (1u << kLat.opp[g.link_dir[i]]))) return false;
  }
  return true;
}

int main() {
  std::mt19937_64 rng(2024);
  std::uniform_real_distribution<double> u01(0.0, 1.0);
  const int shapes[][4] = {{1, 1, 1, 0}, {3, 1, 1, 1}, {1, 6, 3, 1}, {7, 5, 4, 2},
                           {16, 9, 11, 5}, {12, 12, 12, 3}, {20, 18, 9, 8}};
  int failures = 0, cases = 0;
  for (const auto& s : shapes) {
    const int nx = s[0], ny = s[1], nz = s[2], ns = s[3];
    const int emin = std::min(nx, std::min(ny, nz));
    for (int rep = 0; rep < 3; ++rep) {
      std::vector<lbm_sphere> sp(ns);
      for (auto& q : sp) {
        q.cx = u01(rng) * nx;
        q.cy = u01(rng) * ny;
        q.cz = u01(rng) * nz;
        q.r = 0.3 + u01(rng) * 0.45 * emin;
      }
      Geometry g;
      std::string err;
      bool ok;
      if (ns > 0) {
        ok = build_geometry(nullptr, sp.data(), ns, nx, ny, nz, g, err);
      } else {
        std::vector<uint8_t> m((size_t)nx * ny * nz);
        for (auto& v : m) v = u01(rng) < 0.3;
        m[0] = 0;
        ok = build_geometry(m.data(), nullptr, 0, nx, ny, nz, g, err);
      }
      ++cases;
      if (!ok) {
        // an all-solid draw is a legal error; anything else is a failure
        if (err.find("fluid") == std::string::npos) ++failures;
        continue;
      }
      if (!consistent(g)) ++failures;
      Geometry stack;
      append_cell(stack, g);
      append_cell(stack, g);
      if (stack.ncell != 2 * g.ncell || stack.link_cell.size() != 2 * g.link_cell.size()) ++failures;
    }
  }
  std::printf("geometry sanitizer driver: %d cases, %d failures\n", cases, failures);
  return failures ? 1 : 0;
}
