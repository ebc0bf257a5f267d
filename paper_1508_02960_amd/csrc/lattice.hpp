// D3Q19 lattice constants for the GPU library (host and device).
//
// Velocity order is the ABI order documented in include/lbm.h.  Weights are
// the D3Q19 values 1/3, 1/18, 1/36 (Sec. 2 of arXiv:1508.02960: weights
// normalised to unity, cs^2 = 1/3).  The MRT moment basis is the
// d'Humieres D3Q19 set of orthogonal polynomials (eq. (MRT)).
#pragma once
#include <cstdint>

namespace lbm {

constexpr int kQ = 19;

struct Lattice {
  int ex[kQ], ey[kQ], ez[kQ], opp[kQ];
  double w[kQ];
};

constexpr Lattice make_lattice() {
  Lattice L{};
  // rest, 6 axis directions, 12 edge diagonals (xy, xz, yz planes)
  const int v[kQ][3] = {{0, 0, 0},   {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                        {0, 0, 1},   {0, 0, -1}, {1, 1, 0},   {-1, 1, 0}, {1, -1, 0},
                        {-1, -1, 0}, {1, 0, 1},  {-1, 0, 1},  {1, 0, -1}, {-1, 0, -1},
                        {0, 1, 1},   {0, -1, 1}, {0, 1, -1},  {0, -1, -1}};
  for (int k = 0; k < kQ; ++k) {
    L.ex[k] = v[k][0];
    L.ey[k] = v[k][1];
    L.ez[k] = v[k][2];
    const int n2 = v[k][0] * v[k][0] + v[k][1] * v[k][1] + v[k][2] * v[k][2];
    L.w[k] = n2 == 0 ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  for (int k = 0; k < kQ; ++k)
    for (int j = 0; j < kQ; ++j)
      if (v[j][0] == -v[k][0] && v[j][1] == -v[k][1] && v[j][2] == -v[k][2]) L.opp[k] = j;
  return L;
}

constexpr Lattice kLat = make_lattice();

// MRT moment matrix M[i][k] and the squared row norms |M_i|^2.
struct MrtBasis {
  double m[kQ][kQ];
  double n2[kQ];
};

constexpr double mrt_poly(int i, double x, double y, double z) {
  const double e2 = x * x + y * y + z * z;
  switch (i) {
    case 0: return 1.0;
    case 1: return 19.0 * e2 - 30.0;
    case 2: return (21.0 * e2 * e2 - 53.0 * e2 + 24.0) * 0.5;
    case 3: return x;
    case 4: return (5.0 * e2 - 9.0) * x;
    case 5: return y;
    case 6: return (5.0 * e2 - 9.0) * y;
    case 7: return z;
    case 8: return (5.0 * e2 - 9.0) * z;
    case 9: return 3.0 * x * x - e2;
    case 10: return (3.0 * e2 - 5.0) * (3.0 * x * x - e2);
    case 11: return y * y - z * z;
    case 12: return (3.0 * e2 - 5.0) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
  }
}

constexpr MrtBasis make_mrt() {
  MrtBasis B{};
  for (int i = 0; i < kQ; ++i) {
    double s = 0.0;
    for (int k = 0; k < kQ; ++k) {
      B.m[i][k] = mrt_poly(i, kLat.ex[k], kLat.ey[k], kLat.ez[k]);
      s += B.m[i][k] * B.m[i][k];
    }
    B.n2[i] = s;
  }
  return B;
}

constexpr MrtBasis kMrt = make_mrt();

// Per-cell flag word.  Fluid cell: bit k (1..18) set when the pull source
// c - e_k of direction k is solid (a wall link; the slot of that solid source
// in plane k holds the wall coefficient).  Solid cell: kSolid, and bit k set
// when c + e_k is fluid (this cell's slot in plane k is such a link slot).
constexpr uint32_t kSolid = 1u << 31;
constexpr uint32_t kLinkMask = 0x7FFFEu;

}  // namespace lbm
