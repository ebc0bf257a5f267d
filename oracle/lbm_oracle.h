/*
 * FP64 CPU oracle for the D3Q19 lattice Boltzmann method of
 * Fattahi, Waluga, Wohlmuth, Ruede, Manhart, Helmig, "Pore-scale lattice
 * Boltzmann simulation of laminar and turbulent flow through a sphere pack"
 * (arXiv:1508.02960).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Conventions (all lattice units):
 *   - velocity k = 0..18 in the order  0:(0,0,0)
 *       1:(1,0,0) 2:(-1,0,0) 3:(0,1,0) 4:(0,-1,0) 5:(0,0,1) 6:(0,0,-1)
 *       7:(1,1,0) 8:(-1,1,0) 9:(1,-1,0) 10:(-1,-1,0)
 *       11:(1,0,1) 12:(-1,0,1) 13:(1,0,-1) 14:(-1,0,-1)
 *       15:(0,1,1) 16:(0,-1,1) 17:(0,1,-1) 18:(0,-1,-1)
 *   - cell index c = x + nx*(y + ny*z); node (x,y,z) sits at position (x,y,z)
 *   - populations are stored as deviations g_k = f_k - w_k, as an array
 *     g[k*ncell + c] (structure of arrays); solid cells hold zeros
 *   - the domain is periodic in x, y and z; the pressure drop acts along +x
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_SRT = 0, ORC_TRT = 1, ORC_MRT = 2 };
/* Wall rules of Sec. 2.2.1: eq. (noslip), eq. (CLI), eq. (LIBB), eq. (QIBB),
 * eqs. (fstar)-(IEBB) and eq. (MR) (with the (1+q)^2 denominator of kappa_1). */
enum { ORC_SBB = 0, ORC_CLI = 1, ORC_LIBB = 2, ORC_QIBB = 3, ORC_IEBB = 4, ORC_MR = 5 };

typedef struct {
  int32_t nx, ny, nz;
  double tau;       /* 1/omega+, > 1/2 */
  double magic;     /* TRT magic parameter Lambda */
  double drho;      /* density jump across the x-periodic plane */
  int32_t collision;
  int32_t wall;
} orc_params;

/* Lattice: velocities e[3*k+a], weights w[k], opposite direction opp[k]. */
void orc_lattice(int32_t e[57], double w[19], int32_t opp[19]);

/* MRT moment matrix M (row-major 19x19), its inverse and the squared row norms. */
void orc_mrt_matrix(double M[361], double Minv[361], double norm2[19]);

/* Relaxation rates s[19] used for MRT at relaxation time tau. */
void orc_mrt_rates(double tau, double s[19]);

/* TRT omega- from tau and Lambda. */
double orc_trt_omega_minus(double tau, double magic);

/* Deviation equilibrium g^eq_k = f^eq_k(1+drho, u) - w_k. */
void orc_equilibrium(double drho, const double u[3], double geq[19]);

/* Collide one cell in place (input: post-streaming deviations). */
void orc_collide(const orc_params* p, double g[19]);

/* MRT collision with explicit relaxation rates s[19]. */
void orc_collide_mrt_rates(const double s[19], double g[19]);

/* Solid mask from spheres (cx,cy,cz,r per sphere): 1 iff the node lies
 * strictly inside a sphere or one of its periodic images.  Returns #solid. */
int64_t orc_voxelise(int32_t nx, int32_t ny, int32_t nz,
                     const double* spheres, int32_t n_spheres, uint8_t* mask);

/* Normalised wall distance of the link from fluid node (x,y,z) along e_j
 * to the first sphere surface (spheres given), in [0,1]. */
double orc_link_q(int32_t nx, int32_t ny, int32_t nz, const double* spheres,
                  int32_t n_spheres, int32_t x, int32_t y, int32_t z, int32_t j);

/* Dense wall-distance table Q[j*ncell + c]: q of link (c, j) if c is fluid
 * and c + e_j is solid, else -1.  Without spheres every link gets q = 1/2.
 * Returns the number of links. */
int64_t orc_wall_q(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask,
                   const double* spheres, int32_t n_spheres, double* Q);

/* g = g^eq(drho0, u0) on fluid cells, 0 on solid cells.  drho0 (ncell) and
 * u0 (3*ncell, component-major u0[a*ncell + c]) may be NULL (=0). */
void orc_init(const orc_params* p, const uint8_t* mask, const double* drho0,
              const double* u0, double* g);

/* Incoming value of direction k at fluid node (x,y,z) whose pull source
 * x - e_k is solid, given by the domain's wall rule from the stored
 * post-collision state g (deviations). */
double orc_wall_value(const orc_params* p, const uint8_t* mask, const double* Q,
                      const double* g, int32_t x, int32_t y, int32_t z, int32_t k);

/* Threads used by orc_step in an OpenMP build (default 1); the result is
 * the same for any count. */
void orc_set_threads(int32_t n);

/* One fused stream-then-collide step: gout <- step(g). */
void orc_step(const orc_params* p, const uint8_t* mask, const double* Q,
              const double* g, double* gout);

/* n steps; g holds the result, work is scratch of the same size. */
void orc_run(const orc_params* p, const uint8_t* mask, const double* Q,
             double* g, double* work, int64_t n);

/* Per-cell density deviation and velocity of the stored state
 * (u component-major, u[a*ncell + c]); zeros on solid cells. */
void orc_macroscopic(const orc_params* p, const uint8_t* mask, const double* g,
                     double* drho, double* u);

/* Superficial mean velocity: sum of u over fluid cells / (nx ny nz). */
void orc_mean_velocity(const orc_params* p, const uint8_t* mask,
                       const double* g, double U[3]);

/* Momentum-exchange force on the solid, summed over all wall links, from
 * the stored post-collision state g (time t) and the incoming link values
 * it produces at t+1. */
void orc_drag(const orc_params* p, const uint8_t* mask, const double* Q,
              const double* g, double F[3]);

/* Darcy permeability K_D = nu * U * nx / dp with dp = drho/3. */
double orc_permeability(const orc_params* p, double U);

/* Run until the relative change of the superficial U_x over `interval`
 * steps stays below tol for 3 checks in a row.  Returns 0 when converged,
 * 1 when max_steps was reached, 2 on a non-finite or supersonic state. */
int32_t orc_run_to_residual(const orc_params* p, const uint8_t* mask,
                            const double* Q, double* g, double* work, double tol,
                            int64_t max_steps, int64_t interval,
                            int64_t* steps_done, double* residual);

#ifdef __cplusplus
}
#endif
#endif
