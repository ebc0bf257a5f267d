/*
 * FP64 CPU oracle for the D3Q19 lattice Boltzmann method of Fattahi et al.,
 * "Pore-scale lattice Boltzmann simulation of laminar and turbulent flow
 * through a sphere pack" (arXiv:1508.02960).
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against.
 * Plain loops in double precision, written to be checked by eye against the
 * paper; speed is not a goal.  Built with -O2 -ffp-contract=off so that every
 * product is rounded before it is added.
 *
 * Paper passages followed (section / equation of arXiv:1508.02960):
 *   Sec. 2, eq. (LBE) and (collision)/(streaming): stream-then-collide order
 *   eq. (equilibrium): incompressible equilibrium, rho0 = 1, cs^2 = 1/3
 *   eq. (Macro): density and velocity moments
 *   Sec. 2.1 (SRT), eq. (MRT) with Pan's and Khirevich's rates, eq. (TRT)
 *   Sec. 2.2.1, eq. (noslip): simple bounce-back; eq. (CLI)
 *   Sec. 2.2.2, eqs. (generalPeriodicRho)-(PeriodicfunkownRight): periodic
 *     pressure drop
 *   eq. (Darcy) and Sec. 3: permeability, superficial velocity
 * Readings of points the paper leaves open are marked READING in the code.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D3Q19 velocity set (Sec. 2: 19 discrete velocities e_k). */
static const int32_t VEL[19][3] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
    {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, 1, 0},  {1, -1, 0},
    {-1, -1, 0}, {1, 0, 1},  {-1, 0, 1}, {1, 0, -1},  {-1, 0, -1},
    {0, 1, 1},  {0, -1, 1},  {0, 1, -1}, {0, -1, -1}};

/* Weight of a D3Q19 velocity: 1/3 for rest, 1/18 for axis, 1/36 for
 * diagonal directions (the weights are normalised to one, eq. (equilibrium)). */
static double weight_of(int k) {
  int n2 = VEL[k][0] * VEL[k][0] + VEL[k][1] * VEL[k][1] + VEL[k][2] * VEL[k][2];
  if (n2 == 0) return 1.0 / 3.0;
  if (n2 == 1) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

/* The diametrically opposite direction kbar: e_kbar = -e_k. */
static int find_opposite(int k) {
  for (int j = 0; j < 19; ++j)
    if (VEL[j][0] == -VEL[k][0] && VEL[j][1] == -VEL[k][1] &&
        VEL[j][2] == -VEL[k][2])
      return j;
  return -1;
}

/* Tables derived once from VEL (opposites, weights, MRT matrix). */
static int OPP_T[19];
static double W_T[19];
static double M_T[361], MINV_T[361], N2_T[19];
static int tables_ready = 0;
void orc_mrt_matrix(double M[361], double Minv[361], double norm2[19]);
static double weight_of(int k);

static void ensure_tables(void) {
  if (tables_ready) return;
  for (int k = 0; k < 19; ++k) {
    OPP_T[k] = find_opposite(k);
    W_T[k] = weight_of(k);
  }
  orc_mrt_matrix(M_T, MINV_T, N2_T);
  tables_ready = 1;
}

static int opposite_of(int k) {
  ensure_tables();
  return OPP_T[k];
}

void orc_lattice(int32_t e[57], double w[19], int32_t opp[19]) {
  for (int k = 0; k < 19; ++k) {
    for (int a = 0; a < 3; ++a) e[3 * k + a] = VEL[k][a];
    w[k] = weight_of(k);
    opp[k] = opposite_of(k);
  }
}

/* ------------------------------------------------------------------ MRT */

/* Rows of M: the d'Humieres D3Q19 polynomials of the velocity components
 * (eq. (MRT): Gram-Schmidt-orthogonal rows).  Moment order
 *  0 rho, 1 e, 2 eps, 3 jx, 4 qx, 5 jy, 6 qy, 7 jz, 8 qz, 9 3pxx, 10 3pixx,
 *  11 pww, 12 piww, 13 pxy, 14 pyz, 15 pxz, 16 mx, 17 my, 18 mz. */
static double mrt_row(int i, int k) {
  double x = VEL[k][0], y = VEL[k][1], z = VEL[k][2];
  double e2 = x * x + y * y + z * z;
  switch (i) {
    case 0: return 1.0;
    case 1: return 19.0 * e2 - 30.0;
    case 2: return (21.0 * e2 * e2 - 53.0 * e2 + 24.0) / 2.0;
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
    case 18: return (x * x - y * y) * z;
  }
  return 0.0;
}

/* READING: the paper prints R = M^T S M for an "orthogonal" M whose rows are
 * orthogonal but not normalised; the operator meant is M^{-1} S M with
 * M^{-1} = M^T diag(1/|row_i|^2). */
void orc_mrt_matrix(double M[361], double Minv[361], double norm2[19]) {
  for (int i = 0; i < 19; ++i)
    for (int k = 0; k < 19; ++k) M[19 * i + k] = mrt_row(i, k);
  for (int i = 0; i < 19; ++i) {
    double s = 0.0;
    for (int k = 0; k < 19; ++k) s += M[19 * i + k] * M[19 * i + k];
    norm2[i] = s;
  }
  for (int k = 0; k < 19; ++k)
    for (int i = 0; i < 19; ++i) Minv[19 * k + i] = M[19 * i + k] / norm2[i];
}

/* Relaxation rates (Sec. 2.1, MRT paragraph):
 *  conserved moments rho, jx, jy, jz (rows 0,3,5,7): their rate does not
 *    matter because their non-equilibrium part is zero; set to 0 as printed;
 *  viscous modes 9, 11, 13, 14, 15: s_nu = 1/tau = (3 nu + 1/2)^-1;
 *  energy modes 1, 2 (Khirevich's modification): (1/s_nu - 1/2)/(1/s_i - 1/2)
 *    is held at 4.6;
 *  remaining kinetic modes 4, 6, 8, 10, 12, 16, 17, 18 (Pan's choice):
 *    s_zeta = 8 (2 - s_nu) / (8 - s_nu). */
void orc_mrt_rates(double tau, double s[19]) {
  double s_nu = 1.0 / tau;
  double s_e = 1.0 / (0.5 + (tau - 0.5) / 4.6);
  double s_zeta = 8.0 * (2.0 - s_nu) / (8.0 - s_nu);
  for (int i = 0; i < 19; ++i) s[i] = s_zeta;
  s[0] = s[3] = s[5] = s[7] = 0.0;
  s[9] = s[11] = s[13] = s[14] = s[15] = s_nu;
  s[1] = s[2] = s_e;
}

/* ------------------------------------------------------------ collision */

/* TRT: Lambda = (1/omega+ - 1/2)(1/omega- - 1/2) solved for omega-. */
double orc_trt_omega_minus(double tau, double magic) {
  return 1.0 / (0.5 + magic / (tau - 0.5));
}

/* eq. (equilibrium) with rho = 1 + drho, rho0 = 1, cs^-2 = 3, written for
 * the deviation g^eq_k = f^eq_k - w_k: the constant w_k * 1 cancels, leaving
 * w_k {drho + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u} (no subtraction of nearly equal
 * numbers at small drho and u). */
void orc_equilibrium(double drho, const double u[3], double geq[19]) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  ensure_tables();
  for (int k = 0; k < 19; ++k) {
    double eu = VEL[k][0] * u[0] + VEL[k][1] * u[1] + VEL[k][2] * u[2];
    geq[k] = W_T[k] * (drho + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
  }
}

/* eq. (Macro): rho = sum f, u = sum e f (rho0 = 1).  With g = f - w the
 * weights add 1 to rho and nothing to u (sum_k w_k e_k = 0). */
static void moments(const double g[19], double* drho, double u[3]) {
  double r = 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
  for (int k = 0; k < 19; ++k) {
    r += g[k];
    ux += VEL[k][0] * g[k];
    uy += VEL[k][1] * g[k];
    uz += VEL[k][2] * g[k];
  }
  *drho = r;
  u[0] = ux;
  u[1] = uy;
  u[2] = uz;
}

/* eq. (SRT) with R = omega I. */
static void collide_srt(double omega, double g[19]) {
  double drho, u[3], geq[19];
  moments(g, &drho, u);
  orc_equilibrium(drho, u, geq);
  for (int k = 0; k < 19; ++k) g[k] = g[k] - omega * (g[k] - geq[k]);
}

/* eq. (TRT): relax the symmetric part f+ = (f_k + f_kbar)/2 with omega+ and
 * the antisymmetric part f- = (f_k - f_kbar)/2 with omega-; the equilibrium
 * is split the same way. */
static void collide_trt(double wp, double wm, double g[19]) {
  double drho, u[3], geq[19], out[19];
  moments(g, &drho, u);
  orc_equilibrium(drho, u, geq);
  for (int k = 0; k < 19; ++k) {
    int kb = opposite_of(k);
    double fp = 0.5 * (g[k] + g[kb]), fm = 0.5 * (g[k] - g[kb]);
    double ep = 0.5 * (geq[k] + geq[kb]), em = 0.5 * (geq[k] - geq[kb]);
    out[k] = g[k] - wp * (fp - ep) - wm * (fm - em);
  }
  for (int k = 0; k < 19; ++k) g[k] = out[k];
}

/* eq. (MRT) read as g* = g - M^-1 S (M g - M g^eq). */
void orc_collide_mrt_rates(const double s[19], double g[19]) {
  ensure_tables();
  const double* M = M_T;
  const double* Minv = MINV_T;
  double drho, u[3], geq[19], m[19], meq[19], dm[19];
  moments(g, &drho, u);
  orc_equilibrium(drho, u, geq);
  for (int i = 0; i < 19; ++i) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < 19; ++k) {
      a += M[19 * i + k] * g[k];
      b += M[19 * i + k] * geq[k];
    }
    m[i] = a;
    meq[i] = b;
  }
  for (int i = 0; i < 19; ++i) dm[i] = s[i] * (m[i] - meq[i]);
  for (int k = 0; k < 19; ++k) {
    double a = 0.0;
    for (int i = 0; i < 19; ++i) a += Minv[19 * k + i] * dm[i];
    g[k] = g[k] - a;
  }
}

void orc_collide(const orc_params* p, double g[19]) {
  if (p->collision == ORC_SRT) {
    collide_srt(1.0 / p->tau, g);
  } else if (p->collision == ORC_TRT) {
    collide_trt(1.0 / p->tau, orc_trt_omega_minus(p->tau, p->magic), g);
  } else {
    double s[19];
    orc_mrt_rates(p->tau, s);
    orc_collide_mrt_rates(s, g);
  }
}

/* ------------------------------------------------------------- geometry */

static int64_t cell_of(const orc_params* p, int x, int y, int z) {
  return (int64_t)x + (int64_t)p->nx * ((int64_t)y + (int64_t)p->ny * z);
}

/* Periodic index for a coordinate at most one period outside [0, n). */
static int wrap(int i, int n) {
  if (i < 0) return i + n;
  if (i >= n) return i - n;
  return i;
}

/* READING (the paper does not state the voxelisation rule): a node is solid
 * iff it lies strictly inside a sphere, taking periodic images into account
 * (offsets -1, 0, +1 box lengths per axis; radii must be below the box). */
int64_t orc_voxelise(int32_t nx, int32_t ny, int32_t nz, const double* spheres,
                     int32_t n_spheres, uint8_t* mask) {
  int64_t n_solid = 0;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int solid = 0;
        for (int s = 0; s < n_spheres && !solid; ++s) {
          const double* sp = spheres + 4 * s;
          for (int ox = -1; ox <= 1 && !solid; ++ox)
            for (int oy = -1; oy <= 1 && !solid; ++oy)
              for (int oz = -1; oz <= 1 && !solid; ++oz) {
                double dx = x - (sp[0] + ox * nx);
                double dy = y - (sp[1] + oy * ny);
                double dz = z - (sp[2] + oz * nz);
                if (dx * dx + dy * dy + dz * dz < sp[3] * sp[3]) solid = 1;
              }
        }
        mask[(int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z)] =
            (uint8_t)solid;
        n_solid += solid;
      }
  return n_solid;
}

/* Sec. 2.2.1: q = |x_f1 - x_w| / |x_f1 - x_b|.  The wall point is the first
 * crossing of the link segment x + t e_j, t in [0,1], with a sphere surface:
 * the smaller root of |x + t e - c|^2 = r^2. */
double orc_link_q(int32_t nx, int32_t ny, int32_t nz, const double* spheres,
                  int32_t n_spheres, int32_t x, int32_t y, int32_t z,
                  int32_t j) {
  double best = 2.0;
  double e0 = VEL[j][0], e1 = VEL[j][1], e2 = VEL[j][2];
  double a = e0 * e0 + e1 * e1 + e2 * e2;
  for (int s = 0; s < n_spheres; ++s) {
    const double* sp = spheres + 4 * s;
    for (int ox = -1; ox <= 1; ++ox)
      for (int oy = -1; oy <= 1; ++oy)
        for (int oz = -1; oz <= 1; ++oz) {
          double dx = x - (sp[0] + ox * nx);
          double dy = y - (sp[1] + oy * ny);
          double dz = z - (sp[2] + oz * nz);
          double b = 2.0 * (e0 * dx + e1 * dy + e2 * dz);
          double c = dx * dx + dy * dy + dz * dz - sp[3] * sp[3];
          double disc = b * b - 4.0 * a * c;
          if (disc < 0.0) continue;
          double t = (-b - sqrt(disc)) / (2.0 * a);
          if (t >= 0.0 && t <= 1.0 && t < best) best = t;
        }
  }
  return best <= 1.0 ? best : 0.5;
}

int64_t orc_wall_q(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask,
                   const double* spheres, int32_t n_spheres, double* Q) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  int64_t ncell = (int64_t)nx * ny * nz, n_links = 0;
  for (int64_t i = 0; i < 19 * ncell; ++i) Q[i] = -1.0;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int64_t c = cell_of(&p, x, y, z);
        if (mask[c]) continue;
        for (int j = 1; j < 19; ++j) {
          int64_t nb = cell_of(&p, wrap(x + VEL[j][0], nx), wrap(y + VEL[j][1], ny),
                               wrap(z + VEL[j][2], nz));
          if (!mask[nb]) continue;
          Q[j * ncell + c] = n_spheres > 0
                                 ? orc_link_q(nx, ny, nz, spheres, n_spheres, x, y, z, j)
                                 : 0.5;
          ++n_links;
        }
      }
  return n_links;
}

/* ----------------------------------------------------------------- step */

void orc_init(const orc_params* p, const uint8_t* mask, const double* drho0,
              const double* u0, double* g) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  for (int64_t c = 0; c < ncell; ++c) {
    double geq[19] = {0};
    if (!mask[c]) {
      double u[3] = {0.0, 0.0, 0.0}, r = 0.0;
      if (drho0) r = drho0[c];
      if (u0) {
        u[0] = u0[c];
        u[1] = u0[ncell + c];
        u[2] = u0[2 * ncell + c];
      }
      orc_equilibrium(r, u, geq);
    }
    for (int k = 0; k < 19; ++k) g[k * ncell + c] = geq[k];
  }
}

/* Periodic pressure drop (Sec. 2.2.2).  rho_L = rho_R + drho; with the
 * incompressible equilibrium (linear in rho) eqs. (PeriodicFunkown) and
 * (PeriodicFunkownRight) reduce to f_L = f_R + w drho, f_R = f_L - w drho.
 * READING: this is applied to every value that is read across the x-periodic
 * plane, i.e. whose unwrapped x coordinate px lies outside [0, nx): a value
 * taken from the right end to stand on the left (px < 0) gains w drho, a value
 * taken from the left end to stand on the right (px >= nx) loses w drho. */
static double jump(const orc_params* p, int px, int k) {
  ensure_tables();
  if (px < 0) return W_T[k] * p->drho;
  if (px >= p->nx) return -W_T[k] * p->drho;
  return 0.0;
}

static int wrap_any(int i, int n) { return ((i % n) + n) % n; }

/* Value of population k read at the unwrapped node (px, py, pz), with the
 * density jump when the read crosses the x-periodic plane. */
static double read_pop(const orc_params* p, const double* g, int k, int px,
                       int py, int pz) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  int64_t c = cell_of(p, wrap_any(px, p->nx), wrap_any(py, p->ny), wrap_any(pz, p->nz));
  return g[k * ncell + c] + jump(p, px, k);
}

/* Is the node m steps from (x,y,z) along e_k solid? */
static int solid_along(const orc_params* p, const uint8_t* mask, int x, int y, int z,
                       int k, int m) {
  return mask[cell_of(p, wrap_any(x + m * VEL[k][0], p->nx),
                      wrap_any(y + m * VEL[k][1], p->ny),
                      wrap_any(z + m * VEL[k][2], p->nz))] != 0;
}

/* Density deviation and velocity of the stored state at cell c (moments of
 * the post-collision populations, which equal those before collision). */
static void stored_moments(const orc_params* p, const double* g, int64_t c,
                           double* drho, double u[3]) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  *drho = 0.0;
  u[0] = u[1] = u[2] = 0.0;
  for (int k = 0; k < 19; ++k) {
    double v = g[k * ncell + c];
    *drho += v;
    for (int a = 0; a < 3; ++a) u[a] += VEL[k][a] * v;
  }
}

/* Incoming value of direction k at fluid node x = (x,y,z) whose pull source
 * x - e_k is solid.  In the paper's notation the link direction into the
 * wall is k there (j = kbar here), the unknown is f_kbar (f_k here),
 * x_f1 = x, x_f2 = x + e_k and x_f3 = x + 2 e_k (away from the wall), and
 * the right-hand sides are post-collision values at time t_n (the stored
 * state g).  A scheme that needs a node that is solid falls back to the
 * closest scheme with fewer nodes: x_f2 solid -> eq. (noslip) (LIBB and QIBB
 * for q >= 1/2 need x_f1 only and keep LIBB's q >= 1/2 branch); x_f3 solid
 * -> LIBB (from QIBB) or CLI (from MR).  Values read across the x-periodic
 * plane carry the density jump. */
static double wall_value(const orc_params* p, const uint8_t* mask,
                         const double* Q, const double* g, int x, int y, int z,
                         int k) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  int64_t c = cell_of(p, x, y, z);
  int j = opposite_of(k);
  double own_j = g[j * ncell + c];
  if (p->wall == ORC_SBB) return own_j;
  double own_k = g[k * ncell + c];
  double q = Q[j * ncell + c];
  int f2 = !solid_along(p, mask, x, y, z, k, 1);
  int f3 = f2 && !solid_along(p, mask, x, y, z, k, 2);
  int x2 = x + VEL[k][0], y2 = y + VEL[k][1], z2 = z + VEL[k][2];
  int x3 = x + 2 * VEL[k][0], y3 = y + 2 * VEL[k][1], z3 = z + 2 * VEL[k][2];
  int wall = p->wall;
  if (wall == ORC_MR && !f3) wall = ORC_CLI;
  if (wall == ORC_QIBB && (q < 0.5 ? !f3 : !f2)) wall = ORC_LIBB;
  switch (wall) {
    case ORC_CLI: {
      /* eq. (CLI): a = (1 - 2q) / (1 + 2q) */
      if (!f2) return own_j;
      double a = (1.0 - 2.0 * q) / (1.0 + 2.0 * q);
      return a * read_pop(p, g, j, x2, y2, z2) - a * own_k + own_j;
    }
    case ORC_LIBB:
      /* eq. (LIBB) */
      if (q < 0.5) {
        if (!f2) return own_j;
        return (1.0 - 2.0 * q) * read_pop(p, g, j, x2, y2, z2) + 2.0 * q * own_j;
      }
      return (1.0 - 1.0 / (2.0 * q)) * own_k + own_j / (2.0 * q);
    case ORC_QIBB:
      /* eq. (QIBB) */
      if (q < 0.5)
        return q * (1.0 + 2.0 * q) * own_j +
               (1.0 - 4.0 * q * q) * read_pop(p, g, j, x2, y2, z2) -
               q * (1.0 - 2.0 * q) * read_pop(p, g, j, x3, y3, z3);
      return (2.0 * q - 1.0) / q * own_k + own_j / (q * (2.0 * q + 1.0)) +
             (1.0 - 2.0 * q) / (2.0 * q + 1.0) * read_pop(p, g, k, x2, y2, z2);
    case ORC_IEBB: {
      /* eqs. (fstar) and (IEBB): wall velocity u_bf, auxiliary population
       * f*_j(x_b) with the local density deviation of x_f1, and the mixing
       * weight X with omega = 1/tau (omega+ of TRT, s_nu of MRT) */
      double drho1, u1[3], ubf[3], X;
      stored_moments(p, g, c, &drho1, u1);
      if (q < 0.5) {
        double d2;
        if (!f2) return own_j;
        stored_moments(p, g, cell_of(p, wrap_any(x2, p->nx), wrap_any(y2, p->ny),
                                     wrap_any(z2, p->nz)), &d2, ubf);
        X = (2.0 * q - 1.0) / (p->tau - 2.0);
      } else {
        for (int a = 0; a < 3; ++a) ubf[a] = (1.0 - 3.0 / (2.0 * q)) * u1[a];
        X = (2.0 * q - 1.0) / (p->tau + 0.5);
      }
      double eub = 0.0, eu1 = 0.0, uu = 0.0;
      for (int a = 0; a < 3; ++a) {
        eub += VEL[j][a] * ubf[a];
        eu1 += VEL[j][a] * u1[a];
        uu += u1[a] * u1[a];
      }
      double fstar = W_T[j] * (drho1 + 3.0 * eub + 4.5 * eu1 * eu1 - 1.5 * uu);
      return (1.0 - X) * own_j + X * fstar;
    }
    default: {
      /* ORC_MR, eq. (MR); kappa_1 = (1 - 2q - 2q^2)/(1 + q)^2 (the printed
       * (1 + 2q)^2 breaks exactness for linear profiles), kappa_2 = q^2/(1 + q)^2 */
      if (!f2) return own_j;
      double d = (1.0 + q) * (1.0 + q);
      double k1 = (1.0 - 2.0 * q - 2.0 * q * q) / d, k2 = q * q / d;
      return k1 * read_pop(p, g, j, x2, y2, z2) + k2 * read_pop(p, g, j, x3, y3, z3) -
             k1 * own_k - k2 * read_pop(p, g, k, x2, y2, z2) + own_j;
    }
  }
}

double orc_wall_value(const orc_params* p, const uint8_t* mask, const double* Q,
                      const double* g, int32_t x, int32_t y, int32_t z, int32_t k) {
  ensure_tables();
  return wall_value(p, mask, Q, g, x, y, z, k);
}

/* Threads for the time step (OpenMP builds only; 1 by default).  Nodes are
 * updated independently, so the result does not depend on the count. */
static int n_threads = 1;
void orc_set_threads(int32_t n) { n_threads = n > 0 ? n : 1; }

/* Fused step in the paper's order (Sec. 2: first streaming, then collision):
 * pull every population into the node (eq. (streaming) read backwards),
 * replace those whose source is solid by the wall rule, then collide.  Each
 * node reads the old state only and writes its own values, so z planes may be
 * updated by different threads. */
void orc_step(const orc_params* p, const uint8_t* mask, const double* Q,
              const double* g, double* gout) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  ensure_tables();
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(n_threads)
#endif
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        int64_t c = cell_of(p, x, y, z);
        if (mask[c]) {
          for (int k = 0; k < 19; ++k) gout[k * ncell + c] = 0.0;
          continue;
        }
        double loc[19];
        for (int k = 0; k < 19; ++k) {
          int sx = x - VEL[k][0], sy = y - VEL[k][1], sz = z - VEL[k][2];
          int64_t s = cell_of(p, wrap(sx, p->nx), wrap(sy, p->ny), wrap(sz, p->nz));
          if (mask[s])
            loc[k] = wall_value(p, mask, Q, g, x, y, z, k);
          else
            loc[k] = g[k * ncell + s] + jump(p, sx, k);
        }
        orc_collide(p, loc);
        for (int k = 0; k < 19; ++k) gout[k * ncell + c] = loc[k];
      }
}

void orc_run(const orc_params* p, const uint8_t* mask, const double* Q,
             double* g, double* work, int64_t n) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  for (int64_t i = 0; i < n; ++i) {
    orc_step(p, mask, Q, g, work);
    memcpy(g, work, sizeof(double) * 19 * ncell);
  }
}

/* --------------------------------------------------------- observables */

void orc_macroscopic(const orc_params* p, const uint8_t* mask, const double* g,
                     double* drho, double* u) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  for (int64_t c = 0; c < ncell; ++c) {
    double loc[19], r = 0.0, v[3] = {0.0, 0.0, 0.0};
    if (!mask[c]) {
      for (int k = 0; k < 19; ++k) loc[k] = g[k * ncell + c];
      moments(loc, &r, v);
    }
    if (drho) drho[c] = r;
    if (u) {
      u[c] = v[0];
      u[ncell + c] = v[1];
      u[2 * ncell + c] = v[2];
    }
  }
}

/* READING: the velocity in Darcy's law (eq. (Darcy), "volume averaged") is the
 * superficial one, the sum of u over fluid nodes divided by all nodes. */
void orc_mean_velocity(const orc_params* p, const uint8_t* mask,
                       const double* g, double U[3]) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  double s[3] = {0.0, 0.0, 0.0};
  for (int64_t c = 0; c < ncell; ++c) {
    if (mask[c]) continue;
    double loc[19], r, v[3];
    for (int k = 0; k < 19; ++k) loc[k] = g[k * ncell + c];
    moments(loc, &r, v);
    for (int a = 0; a < 3; ++a) s[a] += v[a];
  }
  for (int a = 0; a < 3; ++a) U[a] = s[a] / (double)ncell;
}

/* READING (the paper gives no force formula): momentum exchange summed over
 * the wall links (x, j), j pointing into the solid:
 *   F = sum e_j [ ftilde_j(x, t) + f_kbar(x, t+1) ],  kbar = opposite of j,
 * in absolute populations f = g + w. */
void orc_drag(const orc_params* p, const uint8_t* mask, const double* Q,
              const double* g, double F[3]) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  double s[3] = {0.0, 0.0, 0.0};
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        int64_t c = cell_of(p, x, y, z);
        if (mask[c]) continue;
        for (int j = 1; j < 19; ++j) {
          int64_t nb = cell_of(p, wrap(x + VEL[j][0], p->nx),
                               wrap(y + VEL[j][1], p->ny), wrap(z + VEL[j][2], p->nz));
          if (!mask[nb]) continue;
          int k = opposite_of(j);
          double out = g[j * ncell + c] + weight_of(j);
          double back = wall_value(p, mask, Q, g, x, y, z, k) + weight_of(k);
          for (int a = 0; a < 3; ++a) s[a] += VEL[j][a] * (out + back);
        }
      }
  for (int a = 0; a < 3; ++a) F[a] = s[a];
}

/* eq. (Darcy): K_D = mu U / |grad P| with mu = nu rho0 = nu,
 * nu = (tau - 1/2)/3 (Sec. 2.1), |grad P| = dp / L with L = nx and
 * dp = cs^2 drho = drho / 3 (equation of state p = rho cs^2). */
double orc_permeability(const orc_params* p, double U) {
  double nu = (p->tau - 0.5) / 3.0;
  double dp = p->drho / 3.0;
  return nu * U * p->nx / dp;
}

/* Largest |u| over fluid nodes; non-finite if any node is. */
static double max_speed(const orc_params* p, const uint8_t* mask, const double* g) {
  int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  double m = 0.0;
  for (int64_t c = 0; c < ncell; ++c) {
    if (mask[c]) continue;
    double loc[19], r, v[3];
    for (int k = 0; k < 19; ++k) loc[k] = g[k * ncell + c];
    moments(loc, &r, v);
    double s = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (!isfinite(s) || !isfinite(r)) return INFINITY;
    if (s > m) m = s;
  }
  return m;
}

/* READING of the stopping rule: the paper stops when the time-averaged drag
 * stops changing (Sec. 4); here the relative change of the superficial U_x
 * over `interval` steps must stay below tol for three checks in a row. */
int32_t orc_run_to_residual(const orc_params* p, const uint8_t* mask,
                            const double* Q, double* g, double* work, double tol,
                            int64_t max_steps, int64_t interval,
                            int64_t* steps_done, double* residual) {
  double U[3];
  orc_mean_velocity(p, mask, g, U);
  double prev = U[0], res = INFINITY;
  int64_t done = 0;
  int below = 0, status = 1;
  double cs = 1.0 / sqrt(3.0);
  while (done < max_steps) {
    int64_t n = interval;
    if (done + n > max_steps) n = max_steps - done;
    orc_run(p, mask, Q, g, work, n);
    done += n;
    orc_mean_velocity(p, mask, g, U);
    if (!isfinite(U[0]) || max_speed(p, mask, g) > cs) {
      status = 2;
      break;
    }
    res = U[0] != 0.0 ? fabs(U[0] - prev) / fabs(U[0]) : (U[0] == prev ? 0.0 : INFINITY);
    prev = U[0];
    below = res < tol ? below + 1 : 0;
    if (below >= 3) {
      status = 0;
      break;
    }
  }
  if (steps_done) *steps_done = done;
  if (residual) *residual = res;
  return status;
}
