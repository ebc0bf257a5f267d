/*
 * lbm.h - C ABI of the MI355X (gfx950) D3Q19 lattice Boltzmann hot path for
 * pore-scale flow through sphere packs, after Fattahi et al., "Pore-scale
 * lattice Boltzmann simulation of laminar and turbulent flow through a
 * sphere pack" (arXiv:1508.02960).
 *
 * One library, liblbm.so.  Every entry point returns an lbm_status; nothing
 * throws across the ABI.  A domain is created on the host (geometry, wall
 * links and wall distances are computed once, Sec. 3: "we compute the
 * wall-distances ... only once before the time-stepping loop"), then bound to
 * a caller-owned device workspace and a HIP stream.  The library never
 * allocates device memory: the caller (for instance a torch.uint8 tensor on
 * the GPU) owns the workspace and must keep it alive until lbm_destroy.
 *
 * Lattice and layout (shared with the tests; the order of the 19 velocities
 * is an interface convention):
 *   k  = 0:(0,0,0) 1:(1,0,0) 2:(-1,0,0) 3:(0,1,0) 4:(0,-1,0) 5:(0,0,1)
 *        6:(0,0,-1) 7:(1,1,0) 8:(-1,1,0) 9:(1,-1,0) 10:(-1,-1,0) 11:(1,0,1)
 *        12:(-1,0,1) 13:(1,0,-1) 14:(-1,0,-1) 15:(0,1,1) 16:(0,-1,1)
 *        17:(0,1,-1) 18:(0,-1,-1)
 *   cell c = x + nx*(y + ny*z); node (x,y,z) sits at position (x,y,z).
 *   Host-side population arrays are double g[k*ncell + c] holding the
 *   deviation g_k = f_k - w_k of the post-collision state (w = 1/3, 1/18,
 *   1/36); entries of solid cells are 0.
 *   The box is periodic in x, y and z.  The pressure drop acts along +x
 *   (Sec. 2.2.2): rho_left = rho_right + delta_rho across the x-periodic plane.
 *
 * Threading: calls on one domain must not overlap.  Different domains are
 * independent.  All device work is enqueued on the domain's stream; calls that
 * return host data synchronise that stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_domain_s* lbm_domain;

typedef enum {
  LBM_OK = 0,
  LBM_ERR_INVALID_ARG = 1,   /* bad parameter, pointer or size; nothing changed */
  LBM_ERR_WORKSPACE = 2,     /* workspace missing or smaller than required      */
  LBM_ERR_DEVICE = 3,        /* a HIP call failed (message in lbm_last_error)   */
  LBM_ERR_UNSTABLE = 4,      /* non-finite state or |u| above the sound speed   */
  LBM_ERR_NOT_CONVERGED = 5, /* max_steps reached before the residual test held */
  LBM_ERR_STATE = 6          /* call not valid in the current state             */
} lbm_status;

/* Collision operator, Sec. 2.1: eq. (SRT) with R = omega I, eq. (TRT), eq. (MRT). */
typedef enum { LBM_SRT = 0, LBM_TRT = 1, LBM_MRT = 2 } lbm_collision;

/* Solid-wall rule, Sec. 2.2.1, with the wall distance q of each link:
 * eq. (noslip) simple bounce-back, eq. (CLI) central linear interpolation,
 * eq. (LIBB) linear and eq. (QIBB) quadratic interpolated bounce-back,
 * eqs. (fstar)-(IEBB) interpolation/extrapolation bounce-back (omega = 1/tau
 * in X, the local density deviation in f*; undefined at tau = 2), and
 * eq. (MR) multi-reflection with kappa_1 = (1 - 2q - 2q^2)/(1 + q)^2 (the
 * denominator that makes the rule exact for linear profiles).  A rule that
 * needs a second (third) fluid node along the link where there is none falls
 * back to simple bounce-back (LIBB from QIBB, CLI from MR); LIBB and QIBB
 * with q >= 1/2 need only the first node.  LIBB, QIBB, IEBB and MR need FP32
 * or FP64 storage. */
typedef enum {
  LBM_WALL_SBB = 0,
  LBM_WALL_CLI = 1,
  LBM_WALL_LIBB = 2,
  LBM_WALL_QIBB = 3,
  LBM_WALL_IEBB = 4,
  LBM_WALL_MR = 5
} lbm_wall;

/* Storage precision of the populations (deviations g = f - w).  FP64 computes
 * in double; the others compute in float.  FP16 and BF16 store
 * h_k = sigma g_k / w_k in 16 bits with stochastic rounding (each stored
 * value is the 16-bit neighbour below or above with probability given by the
 * distance, from a counter-based hash of cell, direction and step, so runs
 * stay reproducible); the _RNE variants round to nearest even, which biases
 * slowly varying (Stokes) fields by percents.  Dividing by the
 * weight puts all directions on one scale, and sigma (a power of two, see
 * lbm_info.storage_scale) keeps FP16 values in its normal range.  sigma is
 * chosen when a state is set and, for FP16, moved by exact power-of-two
 * rescaling at the residual checks of lbm_run_to_residual when the largest
 * stored magnitude leaves [2^6, 2^13] (it is set to map the largest
 * magnitude of the state and of delta_rho to 2^10).  Between checks the
 * magnitude may grow 64x before FP16 overflows; lbm_step alone does not
 * rescale.  BF16 keeps sigma = 1.  Reductions are FP64 in every mode.
 * Stochastic-rounding modes launch every step separately (no graph replay),
 * since each step needs its own seed. */
typedef enum {
  LBM_FP64 = 0,
  LBM_FP32 = 1,
  LBM_FP16 = 2,     /* stochastic rounding */
  LBM_BF16 = 3,     /* stochastic rounding */
  LBM_FP16_RNE = 4, /* round to nearest even */
  LBM_BF16_RNE = 5  /* round to nearest even */
} lbm_storage;

/* A sphere in lattice units; spheres and their periodic images may overlap.
 * Radii must be positive and smaller than the smallest box edge. */
typedef struct {
  double cx, cy, cz, r;
} lbm_sphere;

typedef struct {
  int32_t nx, ny, nz;     /* box edge in cells, each >= 1, nx*ny*nz < 2^31,     */
                          /* nx*ny < 2^32 / (19 * value bytes) (padded to whole */
                          /* tiles; the kernels' in-plane offsets are 32-bit)   */
  double tau;             /* relaxation time 1/omega+, > 1/2; nu = (tau-1/2)/3  */
  double magic;           /* TRT Lambda in (0, 3/4] (Sec. 2.1); unused by SRT/MRT */
  double delta_rho;       /* density jump across the x-periodic plane           */
  int32_t collision;      /* lbm_collision                                      */
  int32_t wall;           /* lbm_wall                                           */
  int32_t storage;        /* lbm_storage                                        */
  int32_t check_interval; /* steps between residual checks (0 => 100)           */
} lbm_params;

typedef struct {
  int64_t n_cells;         /* nx*ny*nz                                          */
  int64_t n_fluid;         /* fluid cells                                       */
  int64_t n_links;         /* wall links (fluid cell, direction into solid)     */
  int64_t n_fallback;      /* links whose second fluid node is solid (CLI->SBB) */
  int64_t workspace_bytes; /* device bytes lbm_bind needs                       */
  int64_t state_elems;     /* elements of one device state buffer (19 per cell  */
                           /* address, addresses padded to whole runs)          */
  double nu;               /* kinematic viscosity (tau - 1/2)/3                 */
  double omega_plus;       /* 1/tau                                             */
  double omega_minus;      /* TRT antisymmetric rate from Lambda                */
  int64_t bytes_per_fluid_update; /* algorithmic HBM bytes per fluid-cell update */
  double storage_scale;    /* sigma of 16-bit storage (1 otherwise)             */
  int32_t tile_width;      /* cells: the device buffers' tiles (x extent)       */
  int32_t tile_height;     /* cells: the tiles' y extent (width * height = 64   */
                           /* or 128)                                           */
} lbm_info;

/* Create a domain on the host (no device work).  Sec. 3 / Sec. 2.2.1.
 *   solid_mask : host uint8[nz*ny*nx], 1 = solid, or NULL when spheres given.
 *                With a mask every wall link gets q = 1/2 (CLI == SBB).
 *   spheres    : host array of n_spheres spheres, or NULL/0 with a mask.  A
 *                node is solid iff it lies strictly inside a sphere or one of
 *                its periodic images; q of a link is where the segment from the
 *                fluid node along e_j first meets a sphere surface, in [0,1].
 *   Exactly one of solid_mask and spheres must be given.  Inputs are copied;
 *   the caller may free them after the call.
 * Errors: LBM_ERR_INVALID_ARG for tau <= 1/2, TRT Lambda outside (0, 3/4],
 * non-positive or too large dimensions, no fluid cell, bad sphere radius,
 * unknown enum values, both or neither geometry source.  *out is then NULL. */
lbm_status lbm_create_domain(const uint8_t* solid_mask, const lbm_sphere* spheres,
                             int32_t n_spheres, const lbm_params* params,
                             lbm_domain* out);

/* Sizes and derived constants of a created domain. */
lbm_status lbm_get_info(lbm_domain d, lbm_info* info);

/* Copy the solid mask (uint8[ncell]) to host memory. */
lbm_status lbm_get_mask(lbm_domain d, uint8_t* mask);

/* Copy the wall links to host memory, n_links entries each, sorted by cell
 * then direction: fluid cell index, direction j (1..18) with c + e_j solid,
 * wall distance q (Sec. 2.2.1), and 1 if c - e_j is solid (CLI falls back to
 * bounce-back).  Any pointer may be NULL to skip that array. */
lbm_status lbm_get_links(lbm_domain d, int64_t* cell, int32_t* dir, double* q,
                         uint8_t* fallback);

/* Bind the device workspace and stream, upload geometry, and initialise the
 * fluid at rest (g = 0).  workspace: device pointer, 256-byte aligned, at least
 * info.workspace_bytes; owned by the caller.  stream: a hipStream_t or NULL for
 * the null stream.  May be called again to re-bind (state is re-initialised). */
lbm_status lbm_bind(lbm_domain d, void* workspace, size_t workspace_bytes, void* stream);

/* Set the state to the equilibrium g^eq(drho0, u0) of eq. (equilibrium) on
 * fluid cells.  drho0: host double[ncell] or NULL (0); u0: host
 * double[3*ncell] component-major (u_x block, u_y block, u_z block) or NULL. */
lbm_status lbm_init_equilibrium(lbm_domain d, const double* drho0, const double* u0);

/* Load / read back the full post-collision state (host double[19*ncell],
 * layout above).  Values of solid cells are ignored on load, 0 on read. */
lbm_status lbm_set_state(lbm_domain d, const double* g);
lbm_status lbm_get_state(lbm_domain d, double* g);

/* Enqueue n fused stream-then-collide steps (Sec. 2, eq. (streaming) then
 * eq. (collision)) with the wall rule and the periodic pressure drop.
 * Asynchronous; n = 0 is a no-op. */
lbm_status lbm_step(lbm_domain d, int64_t n);

/* Launch shape of the single-domain step: wavefronts per workgroup (waves:
 * 1, 2, 4, 8 or 16), arranged as waves / rows wavefronts across times `rows`
 * tile rows (rows divides waves), and whether 16-bit storage steps two
 * x-adjacent cells per lane (pairs 1: a wavefront takes two tiles of a tile
 * row) or one (pairs 0: one tile).  Results do not depend on the shape (the
 * stored state is the same bit for bit); only the speed does.  The library
 * picks a shape at lbm_create_domain; this call overrides it (for tuning and
 * tests).  pairs 1 needs FP16/BF16 storage and nx a multiple of the tile
 * width that lbm_get_info reports.  LBM_ERR_INVALID_ARG otherwise, for a
 * shape with more workgroups than the workspace has partial sums for, or for
 * a batch. */
lbm_status lbm_set_step_shape(lbm_domain d, int32_t waves, int32_t rows, int32_t pairs);
lbm_status lbm_get_step_shape(lbm_domain d, int32_t* waves, int32_t* rows, int32_t* pairs);

/* Step until the relative change of the superficial mean velocity U_x over
 * check_interval steps stays below tol for three checks in a row (stopping
 * rule read from Sec. 4).  Returns LBM_OK when converged,
 * LBM_ERR_NOT_CONVERGED at max_steps, LBM_ERR_UNSTABLE on a non-finite state
 * or a speed above 1/sqrt(3) (the domain then rejects lbm_step with
 * LBM_ERR_STATE until re-initialised).  steps_done/residual may be NULL. */
lbm_status lbm_run_to_residual(lbm_domain d, double tol, int64_t max_steps,
                               int64_t* steps_done, double* residual);

/* Density deviation (host double[ncell]) and velocity (host double[3*ncell],
 * component-major) of the current state, eq. (Macro); 0 on solid cells.
 * Either pointer may be NULL. */
lbm_status lbm_macroscopic(lbm_domain d, double* drho, double* u);

/* The same fields in device memory, without a host round trip (e.g. as
 * training targets): fields is a caller-owned device double[4*ncell] laid out
 * as [drho | u_x | u_y | u_z], each block ncell values in cell order.
 * Asynchronous on the domain's stream. */
lbm_status lbm_macroscopic_device(lbm_domain d, double* fields);

/* lbm_init_equilibrium from device fields in the layout of
 * lbm_macroscopic_device (e.g. a predicted warm start).  FP32 and FP64
 * storage only (LBM_ERR_INVALID_ARG otherwise: 16-bit storage picks its
 * scale from the host fields).  Asynchronous on the domain's stream. */
lbm_status lbm_init_equilibrium_device(lbm_domain d, const double* fields);

/* Volume-averaged velocity of eq. (Darcy), taken as the superficial mean
 * U[3] = sum over fluid cells of u / ncell (the U of eqs. (Darcy),
 * (Forchheimer) and (AnalyticForce)), the largest |u| over fluid cells and the
 * total density deviation, reduced in double precision on the device.  Any
 * pointer may be NULL. */
lbm_status lbm_mean_velocity(lbm_domain d, double U[3], double* max_speed,
                             double* total_drho);

/* lbm_mean_velocity for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same kernels and the same results bit for bit, but the
 * reduction's scratch (1024 block partial vectors and the final vector,
 * 65 KB) is a static device array of the library, one per GPU, held until
 * the process ends, instead of a region of the domain's workspace.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine);
 * the first call on a GPU looks up the array's device address.  The scratch
 * need does not depend on the domain size (the reduction runs a fixed grid),
 * so no size is rejected.  Every call on one GPU shares its array: calls that
 * overlap on one GPU (from several threads or streams) race and must be
 * serialised by the caller.  Errors as lbm_mean_velocity, plus
 * LBM_ERR_DEVICE if the array cannot be located. */
lbm_status lbm_mean_velocity_static(lbm_domain d, double U[3], double* max_speed,
                                    double* total_drho);

/* Darcy permeability, eq. (Darcy): K_D = nu U_x nx / dp with dp = delta_rho/3
 * (mu = nu for rho0 = 1, pressure gradient dp/nx); U_x is the superficial
 * velocity (lbm_mean_velocity).  Re_p_per_D = U_x / nu is the pore Reynolds
 * number of Sec. 1 divided by the length scale, so Re_p = Re_p_per_D * D for
 * a sphere diameter D (rho = 1).  Any output pointer may be NULL.
 * Errors: LBM_ERR_STATE when delta_rho is 0 or on a batch. */
lbm_status lbm_permeability(lbm_domain d, double* K_D, double* U_x, double* Re_p_per_D);

/* Drag force F_D on the solid, the force of eq. (AnalyticForce)
 * (C_D = F_D / (6 pi mu U r)), by momentum exchange (host double[3]): the
 * sum over wall links (c, j) of e_j (f~_j(c, t) + f_kbar(c, t+1)),
 * f = g + w, with the incoming value given by the wall rule.  At steady state
 * its x component balances the pressure drop, dp ny nz for a jump plane that
 * lies in fluid. */
lbm_status lbm_drag(lbm_domain d, double F[3]);

/* ------------------------------------------------------------------ batches
 * A batch holds n_cells independent periodic cells of the same nx x ny x nz,
 * each with its own solid geometry, relaxation time, magic parameter and
 * pressure drop.  The cells are stacked along z: host arrays of a batch are
 * laid out as for one domain of nx x ny x (n_cells nz) (cell b occupies z in
 * [b nz, (b+1) nz)), but streaming wraps within each cell.  One launch steps
 * every cell; lbm_run_to_residual tests each cell on the device every
 * check_interval steps and drops converged, unstable or finished cells from
 * later launches, so a run is a replayed graph of kernels with no host
 * decision inside; between replays the host reads the count of running
 * cells and, once it falls to half or less, replays graphs that launch
 * blocks only for the running ones (a device list).  lbm_init_equilibrium, lbm_set_state, lbm_get_state,
 * lbm_macroscopic and lbm_step act on the whole stack; lbm_mean_velocity,
 * lbm_permeability, lbm_drag and lbm_set_delta_rho are per-domain and
 * return LBM_ERR_STATE for a batch (use lbm_batch_results).  Storage must be
 * FP32 or FP64. */
typedef struct {
  double tau;       /* > 1/2 */
  double magic;     /* TRT Lambda in (0, 3/4] */
  double delta_rho; /* density jump across the cell's x-periodic plane */
} lbm_cell_params;

/* Create a batch on the host.  common gives nx, ny, nz (of one cell),
 * collision, wall, storage and check_interval (its tau, magic and delta_rho
 * are ignored).  Geometry per cell: either masks (host uint8, n_cells
 * consecutive cell masks) or spheres with sphere_counts[n_cells] (spheres of
 * cell 0 first, then cell 1, ...; each cell needs at least one).  cells:
 * n_cells parameter records.  Errors as lbm_create_domain, per cell. */
lbm_status lbm_create_batch(int32_t n_cells, const uint8_t* masks, const lbm_sphere* spheres,
                            const int32_t* sphere_counts, const lbm_cell_params* cells,
                            const lbm_params* common, lbm_domain* out);

/* Per-cell results of the last lbm_run_to_residual of a batch (host arrays
 * of n_cells, any may be NULL): superficial velocity (3 per cell) and
 * permeability K_D (eq. (Darcy)) at the cell's last check, steps taken,
 * last residual, and status 0 running / 1 converged / 2 unstable /
 * 3 step limit. */
lbm_status lbm_batch_results(lbm_domain d, double* U, double* K_D, int64_t* steps,
                             double* residual, int32_t* status);

/* Launch shape of the batch step: wavefronts per workgroup (waves, 1..16;
 * each wavefront takes one tile of 64 cells of a z plane, consecutive tiles
 * per workgroup) and z planes per workgroup (zper, a divisor of nz).
 * LBM_ERR_INVALID_ARG otherwise. */
lbm_status lbm_batch_set_shape(lbm_domain d, int32_t waves, int32_t zper);

/* Time every admissible (waves, zper) and solid-write mode (lbm_set_solid_writes)
 * over `steps` steps each (after two warm-up steps) with HIP events on the
 * domain's stream, keep the fastest, and return the shape with its time per
 * step in ms (the mode is read with lbm_get_solid_writes).  The state is
 * reset to rest afterwards. */
lbm_status lbm_batch_autotune(lbm_domain d, int32_t steps, int32_t* waves, int32_t* zper,
                              double* ms_per_step);

/* Which solid cells a batch step writes; an implementation choice with no
 * effect on results (fluid cells and wall-link slots hold the same values in
 * every mode), only on speed.  Where a sphere surface cuts a 128-byte line of
 * a direction plane, the fluid cells write only part of it; solid cells
 * sharing the line can complete it (zeros, and copies of their wall-link
 * slots).  mode 0: fluid cells only (default); 1: also solid cells whose
 * 64-cell tile (wavefront) holds a fluid cell; 2: also solid cells whose
 * line holds a fluid cell.  lbm_batch_autotune picks the fastest.  Invalid
 * mode: LBM_ERR_INVALID_ARG; mode 1 or 2 on a single domain (whose step
 * always writes fluid cells only): LBM_ERR_STATE. */
lbm_status lbm_set_solid_writes(lbm_domain d, int32_t mode);
lbm_status lbm_get_solid_writes(lbm_domain d, int32_t* mode);

/* Change the pressure drop of a bound domain (state kept). */
lbm_status lbm_set_delta_rho(lbm_domain d, double delta_rho);

/* Wait for the domain's stream. */
lbm_status lbm_synchronize(lbm_domain d);

/* Release host memory of the domain (the workspace stays the caller's). */
lbm_status lbm_destroy(lbm_domain d);

/* ---------------------------------------------------------------- probes
 * Attainable-bandwidth probes, a measurement aid (not an operation of the
 * method): plain streaming kernels of known byte counts that bound what the
 * step kernel can reach on the GPU at hand and calibrate HBM byte counters.
 * Asynchronous on `stream` (a hipStream_t or NULL); the caller times them,
 * e.g. with events on that stream.  Buffers are caller-owned device memory,
 * 16-byte aligned.
 *   LBM_PROBE_READ     reads n bytes of src (dst: >= 16 bytes, written only
 *                      if the data sum to a sentinel value, i.e. never for
 *                      ordinary data); n a positive multiple of 16
 *   LBM_PROBE_WRITE    writes n bytes to dst (src unused)
 *   LBM_PROBE_COPY     copies n bytes from src to dst
 *   LBM_PROBE_GATHER19 the step's pull pattern on an all-fluid periodic cube
 *                      of edge n (multiple of 16, at most 1024): src and dst
 *                      hold 19 FP32 values for each of n^3 cells in 16 x 4
 *                      tiles, each tile's values as 19 runs of 64 (one per
 *                      direction); reads and writes 2 * 76 n^3 bytes
 * Errors: LBM_ERR_INVALID_ARG for an unknown kind, a bad size, NULL or
 * misaligned buffers; LBM_ERR_DEVICE if the launch fails. */
typedef enum {
  LBM_PROBE_READ = 0,
  LBM_PROBE_WRITE = 1,
  LBM_PROBE_COPY = 2,
  LBM_PROBE_GATHER19 = 3
} lbm_probe_kind;
lbm_status lbm_bandwidth_probe(int32_t kind, const void* src, void* dst, int64_t n,
                               void* stream);

const char* lbm_status_string(lbm_status s);
/* Last error message of the domain ("" if none); NULL domain: last create error. */
const char* lbm_last_error(lbm_domain d);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
