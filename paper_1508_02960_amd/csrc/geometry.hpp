// Host-side geometry of a periodic sphere-pack domain: solid mask, wall
// links with their wall distances q (Sec. 2.2.1 of arXiv:1508.02960), and the
// per-cell flag words the step kernel reads.  Computed once per domain
// (Sec. 3: wall distances are precomputed before time stepping).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "lbm.h"

namespace lbm {

struct Geometry {
  int nx = 0, ny = 0, nz = 0;
  int nz_cell = 0;  // z period: nz for one domain, the cell edge for a batch
  int64_t ncell = 0, n_fluid = 0, n_fallback = 0;
  std::vector<uint8_t> mask;    // 1 = solid
  std::vector<uint32_t> flags;  // see lattice.hpp
  // wall links (fluid cell, direction j into the solid), sorted by cell, dir
  std::vector<int64_t> link_cell;
  std::vector<int32_t> link_dir;
  std::vector<double> link_q;
  std::vector<uint8_t> link_fallback;  // 1 if cell - e_j is solid
};

// Fill g from either a mask or spheres.  Returns false with a message on a
// geometry error (no fluid cell, bad sphere).
bool build_geometry(const uint8_t* mask, const lbm_sphere* spheres, int n_spheres, int nx,
                    int ny, int nz, Geometry& g, std::string& err);

// Append cell geometry `c` (one periodic cell) to the stacked batch `g`
// (cells stacked along z).
void append_cell(Geometry& g, const Geometry& c);

}  // namespace lbm
