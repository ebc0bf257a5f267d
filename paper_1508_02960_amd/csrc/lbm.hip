// C ABI of the D3Q19 hot path (include/lbm.h): domain lifetime, workspace
// layout, kernel launches and host-side control of the time loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "geometry.hpp"
#include "kernels.hpp"
#include "lbm.h"
#include "step_table.hpp"

#define LBM_API extern "C" __attribute__((visibility("default")))

using namespace lbm;

struct lbm_domain_s {
  lbm_params p{};
  Geometry geo;
  std::string err;
  // derived
  long long state_elems = 0;  // elements of one state buffer (19 per address, whole runs)
  size_t elem = 0;       // bytes per stored population
  Tiling tiling{};       // tiled cell order of the device buffers
  long long naddr = 0;   // device cell addresses (cells plus tile padding)
  long long cell_addrs = 0;  // addresses per z period (one batch cell, or the box)
  int waves = 16;        // wavefronts per step workgroup
  int rows = 1;          // tile rows per step workgroup (waves / rows units across)
  bool streaming = false;  // non-temporal stores in the step kernels
  bool pairs = false;      // 16-bit storage: two cells per lane (step_pair_kernel)
  double nu = 0, omega_p = 0, omega_m = 0, s_e = 0, s_zeta = 0;
  double sigma = 1.0;    // 16-bit storage scale (h = sigma g / w), a power of two
  uint64_t step_count = 0;  // steps launched (seeds stochastic rounding)
  // device (inside the caller's workspace)
  bool bound = false;
  bool unstable = false;
  int device = 0;  // GPU holding the workspace
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  void* buf[2] = {nullptr, nullptr};
  int cur = 0;  // buf[cur] holds the current state
  uint32_t* flags = nullptr;
  uint8_t* cls = nullptr;  // class byte per cell (kClsSolid, kClsLinks, kClsNearWall)
  void* side[2] = {nullptr, nullptr};  // IEBB: near-wall velocities of buf[0], buf[1]
  long long* link_slot = nullptr;
  double* link_coef = nullptr;
  double* partials = nullptr;   // per-block partial sums
  double* partials2 = nullptr;  // second-stage partial sums
  long long n_partials = 0;     // capacity of partials (vectors)
  double* result = nullptr;
  double* stage = nullptr;
  size_t stage_cells = 0;  // cells per staging chunk (4 doubles each)
  // replayable launch sequences: kGraphSteps steps starting from buffer p
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  // batches of independent cells (0: one domain)
  int batch = 0;
  long long cell_size = 0;            // cells per batch cell
  std::vector<lbm_cell_params> cellp;  // per-cell tau, Lambda, delta_rho
  int bby = 0, zper = 1;              // batch launch shape: wavefronts (tiles) per block, z planes per block
  int solid_writes = 0;               // which solid cells store (StepParams::solid_writes)
  StepParams* d_cells = nullptr;
  int* d_active = nullptr;      // cells stepped in a residual run
  int* d_active_all = nullptr;  // all ones, for lbm_step
  CellStatus* d_status = nullptr;
  double* d_results = nullptr;
  int* d_nactive = nullptr;     // running cells (count of d_list)
  int* d_list = nullptr;        // the running cells in order (batch_check_kernel)
  std::vector<CellStatus> status_host;
  // layout offsets
  size_t off_buf[2] = {0, 0}, off_flags = 0, off_cls = 0, off_slot = 0, off_coef = 0, off_part = 0,
         off_part2 = 0, off_res = 0, off_stage = 0, off_cells = 0, off_active = 0,
         off_active_all = 0, off_status = 0, off_results = 0, off_nactive = 0, off_list = 0,
         off_side[2] = {0, 0},
         side_bytes = 0, total = 0;
};

namespace {

std::string g_create_error;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

lbm_status fail(lbm_domain d, lbm_status s, const std::string& msg) {
  if (d) d->err = msg;
  return s;
}

#define HIP_OK(d, call)                                                                 \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail((d), LBM_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Call f with a value of the storage type of the domain.
template <class F>
decltype(auto) with_storage(int storage, F&& f) {
  switch (storage) {
    case LBM_FP64: return f(double{});
    case LBM_FP32: return f(float{});
    case LBM_FP16: return f(fp16s_t{});
    case LBM_BF16: return f(bf16s_t{});
    case LBM_FP16_RNE: return f(fp16_t{});
    default: return f(bf16_t{});
  }
}

size_t storage_bytes(int storage) {
  return storage == LBM_FP64 ? 8 : (storage == LBM_FP32 ? 4 : 2);
}
bool is_fp16(int storage) { return storage == LBM_FP16 || storage == LBM_FP16_RNE; }
bool is_stochastic(int storage) { return storage == LBM_FP16 || storage == LBM_BF16; }

// 16-bit storage keeps max_k |g_k| / w_k * sigma inside [kScaleLow, kScaleHigh]
// (FP16 holds up to 65504, a growth of 64x from kScaleTarget between two
// checks; its relative precision is the same from 2^-14 up).
constexpr double kScaleTarget = 1024.0, kScaleHigh = 8192.0, kScaleLow = 64.0;

// Power-of-two sigma that maps magnitude m to about kScaleTarget.
double pick_sigma(double m) {
  if (!(m > 0.0) || !std::isfinite(m)) return kScaleTarget;
  return std::ldexp(1.0, (int)std::floor(std::log2(kScaleTarget / m)));
}

// Tiles of 2^tile_log2 cells (64 or 128), 2^tw_log2 wide.  Compact tiles
// for states beyond the last-level cache (512^3 sphere pack, FP32 CLI: 16 x 4
// tiles 2.51 ms per step against 2.56 ms for 8 x 8 tiles and 2.98 ms for
// rows); 64 x 1 tiles (rows) for smaller states, which stay largely in the
// 256 MB cache and where rows step fastest (128^3, FP32: 54 us against 62 us
// for 16 x 4).
Tiling make_tiling(int nx, int ny, int tw_log2, int tile_log2) {
  Tiling t{};
  t.nx = nx;
  t.ny = ny;
  t.tw_log2 = tw_log2;
  t.th_log2 = tile_log2 - t.tw_log2;
  t.ntx = (nx + (1 << t.tw_log2) - 1) >> t.tw_log2;
  t.nty = (ny + (1 << t.th_log2) - 1) >> t.th_log2;
  t.plane = (t.ntx * t.nty) << tile_log2;
  return t;
}

// Step workgroups: waves / rows wavefronts across times `rows` tile rows of
// one z plane; a wavefront takes a unit of a tile row (one tile, or two
// x-adjacent tiles with two cells per lane).
int step_units_per_row(lbm_domain d) {
  const int row = d->tiling.ntx << d->tiling.tile_log2();  // addresses per tile row
  return d->pairs ? (row + 127) / 128 : row / 64;
}
int step_nbx(lbm_domain d) {
  const int bw = d->waves / d->rows;
  return (step_units_per_row(d) + bw - 1) / bw;
}
dim3 step_block(lbm_domain d) { return dim3(64, d->waves, 1); }
dim3 step_grid(lbm_domain d) {
  const int nby = (d->tiling.nty + d->rows - 1) / d->rows;
  return dim3(step_nbx(d), nby, d->geo.nz);
}

// Non-temporal stores pay once the two state buffers are well beyond the
// 256 MB last-level cache (measured: 15% faster at 256^3 FP32, 2.5 GB;
// 1.6% slower at 128^3, 0.32 GB, where much of the state stays cached).
constexpr size_t kStreamingBytes = size_t(1) << 30;

// IEBB on one domain keeps the velocity of the cells next to its wall links
// in a side buffer per state (StepParams::side_in / side_out); batches sum
// the stored values instead.
bool uses_side(lbm_domain d) { return d->p.wall == LBM_WALL_IEBB && !d->batch; }

void layout(lbm_domain d) {
  d->elem = storage_bytes(d->p.storage);
  // large states: compact tiles and streaming stores (sizes estimated on the
  // unpadded cell count; padding adds at most a few percent)
  d->streaming = 2 * (size_t)kQ * (size_t)d->geo.ncell * d->elem > kStreamingBytes;
  // compact tiles 16 x 4; the 16-bit formats' tiles are 32 cells wide (a
  // 16-lane DPP row of the two-cell lanes is then one tile row).  Batches
  // take 8 x 8: a 128-byte line is then an 8 x 4 patch, which the walls of
  // small pores cut less often (line model of the 128^3 packs of 8-27
  // spheres: 1.18-1.28x the algorithmic lines against 1.29-1.44x), and
  // their step is faster (16 packs of 128^3: 0.617 against 0.668 ms; 256
  // cells of 64^3: 1.568 against 1.611 ms; the states are identical)
  const int tw = d->streaming ? (d->elem == 2 ? 5 : (d->batch ? 3 : 4)) : 6;
  // two cells per lane: 16-bit storage beyond the last-level cache (512^3
  // sphere pack, FP16: 1.68 ms per step against 1.73 ms for one cell per
  // lane; 128^3, in the cache: 36 us against 34 us, so not there), one
  // domain (batches step one cell per lane), the box's x edge on a tile edge
  const bool pairs = d->elem == 2 && d->streaming && !d->batch && d->geo.nx % (1 << tw) == 0;
  // then tiles of 32 x 4 cells, one per wavefront: a +-y pull shares its
  // tile's lines except for one row in four, against one in two for 32 x 2
  // tiles (512^3 sphere pack, FP16: 1.54 ms per step with 4 wavefronts per
  // workgroup against 1.58 ms for pairs of 32 x 2 tiles; all fluid 2.02
  // against 2.17 ms; 32 x 8 tiles 1.79 and 1.95 ms)
  d->tiling = make_tiling(d->geo.nx, d->geo.ny, tw, pairs ? 7 : 6);
  d->pairs = pairs;
  // FP32 and FP64 states of one domain are cut into runs of 128 addresses:
  // every z plane starts on a run (the step kernels split an address into a
  // wavefront-uniform plane part and a 32-bit in-plane part), so a plane of
  // an odd number of tiles gets one tile of padding
  if (d->elem != 2 && !d->batch && d->tiling.plane % (1 << kStepRunLog2)) d->tiling.plane += 64;
  d->cell_addrs = (long long)d->tiling.plane * d->geo.nz_cell;
  d->naddr = (long long)d->tiling.plane * d->geo.nz;
  const int64_t n = d->naddr;
  // State runs (Tiling::slot).  512^3 sphere pack, ms per step: FP32 in
  // runs of 128 addresses 2.37, of 64 2.40, of 256 2.40, in direction
  // planes 2.50; FP16 (two cells per lane) in planes 1.65, in runs of 128
  // to 4096 addresses 1.80-1.83.  Batch cells start on a run (runs of 64).
  if (d->elem == 2 && !d->batch) {
    d->tiling.run_log2 = 40;  // one run: direction planes
    // planes padded so that the 19 streams do not start on the same HBM
    // channel: the address count rounded up to 1024, plus 512
    d->tiling.run_pitch = ((n + 1023) / 1024) * 1024 + 512;
    d->state_elems = (long long)kQ * d->tiling.run_pitch;
  } else {
    d->tiling.run_log2 = d->batch ? kBatchRunLog2 : kStepRunLog2;
    d->tiling.run_pitch = 1LL << d->tiling.run_log2;
    const long long run = d->tiling.run_pitch;
    d->state_elems = (long long)kQ * ((n + run - 1) / run * run);
  }
  // 8 wavefronts (16 x 4 tiles: 128 x 4 cells) with compact tiles, 4 with
  // two cells per lane (32 x 4 tiles: 128 x 4 cells), 4 (256 cells of a row)
  // with rows; never more than a plane has work for
  d->waves = d->streaming ? (d->pairs ? 4 : 8) : 4;
  const int units = step_units_per_row(d);
  d->rows = 1;
  while (d->waves / d->rows > units && d->rows < d->tiling.nty) d->rows *= 2;
  while (d->waves > d->rows && d->waves / d->rows > units) d->waves /= 2;
  static_assert(16 * 64 <= kStepThreads, "step workgroups exceed the kernel's launch bound");
  size_t o = 0;
  const size_t bufb = align256((size_t)d->state_elems * d->elem);
  d->off_buf[0] = o;
  o += bufb;
  d->off_buf[1] = o;
  o += bufb;
  d->off_flags = o;
  o += align256((size_t)n * 4);
  d->off_cls = o;
  o += align256((size_t)n);
  const size_t nl = d->geo.link_cell.size();
  d->off_slot = o;
  o += align256(std::max<size_t>(nl, 1) * 8);
  d->off_coef = o;
  o += align256(std::max<size_t>(nl, 1) * 8);
  // partial sums: room for the step shapes of lbm_set_step_shape with at
  // least two wavefronts per workgroup (about tiles / 2 blocks per plane)
  const dim3 sg = step_grid(d);
  const long long half_row = ((d->tiling.ntx << (d->tiling.tile_log2() - 6)) + 1) / 2;
  d->n_partials = std::max<long long>(kRedBlocks, (long long)sg.x * sg.y * sg.z);
  d->n_partials =
      std::max<long long>(d->n_partials, half_row * d->tiling.nty * (long long)d->geo.nz);
  if (d->batch) {
    // most blocks: one tile and one z plane per block
    d->n_partials = std::max<long long>(
        d->n_partials, (long long)d->tiling.ntx * d->tiling.nty * d->geo.nz);
  }
  d->off_part = o;
  o += align256((size_t)d->n_partials * kRedVals * 8);
  d->off_part2 = o;
  o += align256((size_t)kRedThreads * kRedVals * 8);
  d->off_res = o;
  o += align256(kRedVals * 8);
  // staging: at least one z-plane of cells, at least 1M cells, 4 doubles each
  d->stage_cells = std::max<size_t>((size_t)d->geo.nx * d->geo.ny, size_t(1) << 20);
  d->stage_cells = std::min<size_t>(d->stage_cells, (size_t)n);
  d->off_stage = o;
  o += align256(d->stage_cells * 4 * 8);
  const size_t nb = (size_t)std::max(d->batch, 1);
  d->off_cells = o;
  o += align256(nb * sizeof(StepParams));
  d->off_active = o;
  o += align256(nb * sizeof(int));
  d->off_active_all = o;
  o += align256(nb * sizeof(int));
  d->off_status = o;
  o += align256(nb * sizeof(CellStatus));
  d->off_results = o;
  o += align256(nb * kRedVals * sizeof(double));
  d->off_nactive = o;
  o += align256(sizeof(int));
  d->off_list = o;
  o += align256(nb * sizeof(int));
  // IEBB on one domain: 4 values of the compute type per address and state
  d->side_bytes = uses_side(d) ? (size_t)n * 4 * (d->elem == 8 ? 8 : 4) : 0;
  for (int i = 0; i < 2; ++i) {
    d->off_side[i] = o;
    o += align256(d->side_bytes);
  }
  d->total = o;
}

// The in-plane part of a state byte offset (state_lane) fits in 32 bits.
bool plane_offsets_fit(lbm_domain d) {
  const int64_t per_address = d->elem == 2 ? 2 : (int64_t)kQ * d->elem;
  return per_address * d->tiling.plane < (int64_t(1) << 32);
}

// Cells of one z period in row-major host order (one batch cell, or the box).
long long cell_cells(lbm_domain d) { return (long long)d->geo.nx * d->geo.ny * d->geo.nz_cell; }

// The FP32 copies of a StepParams' rates and jumps, and the 16-bit formats'
// factors between stored values h and deviations g (h = sigma g / w_k) per
// weight class.
void set_float_params(StepParams& sp) {
  const double w[3] = {kLat.w[0], kLat.w[1], kLat.w[7]};
  for (int i = 0; i < 3; ++i) {
    sp.dec[i] = (float)(w[i] * (1.0 / sp.sigma));
    sp.enc[i] = (float)(sp.sigma / w[i]);
  }
  sp.omega_pf = (float)sp.omega_p;
  sp.omega_mf = (float)sp.omega_m;
  sp.s_ef = (float)sp.s_e;
  sp.s_zetaf = (float)sp.s_zeta;
  sp.jump_axisf = (float)sp.jump_axis;
  sp.jump_diagf = (float)sp.jump_diag;
}

StepParams step_params(lbm_domain d) {
  StepParams sp;
  sp.t = d->tiling;
  sp.nx = d->geo.nx;
  sp.ny = d->geo.ny;
  sp.nz = d->geo.nz;
  sp.jump_axis = (1.0 / 18.0) * d->p.delta_rho;
  sp.jump_diag = (1.0 / 36.0) * d->p.delta_rho;
  sp.omega_p = d->omega_p;
  sp.omega_m = d->omega_m;
  sp.s_e = d->s_e;
  sp.s_zeta = d->s_zeta;
  sp.sigma = d->sigma;
  set_float_params(sp);
  sp.wall = d->p.wall;
  sp.solid_writes = d->solid_writes;
  sp.side_in = d->side[d->cur];
  sp.side_out = d->side[1 - d->cur];
  sp.bw = std::max(1, d->waves / std::max(1, d->rows));
  sp.bh = std::max(1, d->rows);
  sp.nbx = d->batch ? 1 : step_nbx(d);
  sp.seed = hash32((uint32_t)d->step_count ^ hash32((uint32_t)(d->step_count >> 32) + 0x5bd1e995u));
  return sp;
}

// Wall template of a rule: SBB and CLI have their own, the other
// interpolated rules share the general one (FP32/FP64 storage only).
int wall_template(int wall) { return wall <= LBM_WALL_CLI ? wall : kGEN; }

const void* step_function(lbm_domain d, bool red) {
  return with_storage(d->p.storage, [&](auto tag) -> const void* {
    using S = decltype(tag);
    return step_kernel_entry<S>(red, d->streaming, d->pairs, d->p.collision,
                                wall_template(d->p.wall));
  });
}

// Steps replayed as one graph launch (an even count keeps the buffer parity).
constexpr int kGraphSteps = 32;

void drop_graphs(lbm_domain d) {
  for (int i = 0; i < 2; ++i) {
    if (d->graph_exec[i]) (void)hipGraphExecDestroy(d->graph_exec[i]);
    if (d->graph[i]) (void)hipGraphDestroy(d->graph[i]);
    d->graph_exec[i] = nullptr;
    d->graph[i] = nullptr;
  }
}

// One step launch from buffer d->cur; red adds the block partial sums.
lbm_status launch_step(lbm_domain d, bool red) {
  StepParams sp = step_params(d);
  const void* src = d->buf[d->cur];
  void* dst = d->buf[1 - d->cur];
  const uint8_t* cl = d->cls;
  uint32_t* fl = d->flags;
  double* part = d->partials;
  void* args[] = {(void*)&src, (void*)&dst, (void*)&cl, (void*)&fl, (void*)&sp, (void*)&part};
  const dim3 grid = step_grid(d), block = step_block(d);
  HIP_OK(d, hipLaunchKernel(step_function(d, red), grid, block, args, 0, d->stream));
  d->cur = 1 - d->cur;
  ++d->step_count;
  return LBM_OK;
}

// Build the graph of kGraphSteps plain steps starting from buffer `from`:
// kernel nodes only, each depending on the previous one.
lbm_status build_graph(lbm_domain d, int from) {
  hipGraph_t g = nullptr;
  HIP_OK(d, hipGraphCreate(&g, 0));
  StepParams sp = step_params(d);
  const uint8_t* cl = d->cls;
  uint32_t* fl = d->flags;
  double* part = d->partials;
  const dim3 grid = step_grid(d), block = step_block(d);
  const void* fn = step_function(d, false);
  hipGraphNode_t prev = nullptr;
  for (int i = 0; i < kGraphSteps; ++i) {
    const void* src = d->buf[(from + i) & 1];
    void* dst = d->buf[(from + i + 1) & 1];
    sp.side_in = d->side[(from + i) & 1];
    sp.side_out = d->side[(from + i + 1) & 1];
    void* args[] = {(void*)&src, (void*)&dst, (void*)&cl, (void*)&fl, (void*)&sp, (void*)&part};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(fn);
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(d, LBM_ERR_DEVICE, std::string("hipGraphAddKernelNode: ") + hipGetErrorString(e));
    }
    prev = node;
  }
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(d, LBM_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  d->graph[from] = g;
  d->graph_exec[from] = ex;
  return LBM_OK;
}

lbm_status enqueue_steps(lbm_domain d, int64_t n) {
  // stochastic rounding needs a fresh seed per step: plain launches only
  while (n >= kGraphSteps && !is_stochastic(d->p.storage)) {
    if (!d->graph_exec[d->cur]) {
      lbm_status st = build_graph(d, d->cur);
      if (st != LBM_OK) return st;
    }
    HIP_OK(d, hipGraphLaunch(d->graph_exec[d->cur], d->stream));
    n -= kGraphSteps;  // even count: d->cur unchanged
  }
  for (int64_t i = 0; i < n; ++i) {
    lbm_status st = launch_step(d, false);
    if (st != LBM_OK) return st;
  }
  HIP_OK(d, hipGetLastError());
  return LBM_OK;
}

// ---- batches

dim3 batch_block(lbm_domain d) { return dim3(64, d->bby, 1); }
// Grid over `slots` cells (all of them by default): tile blocks times z
// blocks of each cell.
dim3 batch_grid(lbm_domain d, int slots = -1) {
  const int tiles = d->tiling.ntx * d->tiling.nty;
  if (slots < 0) slots = d->batch;
  return dim3((tiles + d->bby - 1) / d->bby, 1,
              (unsigned)((long long)slots * d->geo.nz_cell / d->zper));
}

const void* batch_function(lbm_domain d, bool red) {
  const int wt = wall_template(d->p.wall);
  if (d->p.storage == LBM_FP64)
    return batch_kernel_entry<double>(red, d->streaming, d->p.collision, wt);
  return batch_kernel_entry<float>(red, d->streaming, d->p.collision, wt);
}

// Kernel-node or launch arguments of one batch step from buffer `from`.
struct BatchArgs {
  const void* src;
  void* dst;
  const uint8_t* cls;
  const uint32_t* flags;
  const StepParams* cells;
  const int* active;
  const int* list;
  const int* n_list;
  int nz_cell;
  long long cell_size;
  int zper;
  double* partials;
  void* ptrs[12];
  // listed: the grid runs over d_list's cells (batch runs), else over all
  void fill(lbm_domain d, int from, const int* act, bool listed) {
    src = d->buf[from];
    dst = d->buf[1 - from];
    cls = d->cls;
    flags = d->flags;
    cells = d->d_cells;
    active = act;
    list = listed ? d->d_list : nullptr;
    n_list = listed ? d->d_nactive : nullptr;
    nz_cell = d->geo.nz_cell;
    cell_size = d->cell_addrs;
    zper = d->zper;
    partials = d->partials;
    ptrs[0] = &src;
    ptrs[1] = &dst;
    ptrs[2] = &cls;
    ptrs[3] = &flags;
    ptrs[4] = &cells;
    ptrs[5] = &active;
    ptrs[6] = &list;
    ptrs[7] = &n_list;
    ptrs[8] = &nz_cell;
    ptrs[9] = &cell_size;
    ptrs[10] = &zper;
    ptrs[11] = &partials;
  }
};

lbm_status launch_batch_step(lbm_domain d, bool red, const int* act) {
  BatchArgs a;
  a.fill(d, d->cur, act, false);
  HIP_OK(d, hipLaunchKernel(batch_function(d, red), batch_grid(d), batch_block(d), a.ptrs, 0,
                            d->stream));
  d->cur = 1 - d->cur;
  ++d->step_count;
  return LBM_OK;
}

lbm_status enqueue_batch_steps(lbm_domain d, int64_t n) {
  for (int64_t i = 0; i < n; ++i) {
    lbm_status st = launch_batch_step(d, false, d->d_active_all);
    if (st != LBM_OK) return st;
  }
  HIP_OK(d, hipGetLastError());
  return LBM_OK;
}

// Graph of `reps` check intervals of `interval` steps starting from buffer
// `from`: (interval - 1) steps, one step with block partials, the per-cell
// fold and the device-side convergence test.  Kernel nodes only.  The steps
// run over `slots` entries of the list of running cells.
lbm_status build_batch_graph(lbm_domain d, int from, int reps, int interval, double tol,
                             long long max_steps, int slots, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIP_OK(d, hipGraphCreate(&g, 0));
  hipGraphNode_t prev = nullptr;
  auto add = [&](const void* fn, dim3 grid, dim3 block, void** args) -> hipError_t {
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(fn);
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    if (e == hipSuccess) prev = node;
    return e;
  };
  const dim3 grid = batch_grid(d, slots), block = batch_block(d);
  const long long blocks_per_cell =
      (long long)grid.x * grid.y * ((long long)d->geo.nz_cell / d->zper);  // grid.y is 1
  int parity = from;
  hipError_t e = hipSuccess;
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    for (int i = 0; i < interval && e == hipSuccess; ++i) {
      const bool red = i == interval - 1;
      BatchArgs a;
      a.fill(d, parity, d->d_active, true);
      e = add(batch_function(d, red), grid, block, a.ptrs);
      parity = 1 - parity;
    }
    if (e != hipSuccess) break;
    const double* part = d->partials;
    long long bpc = blocks_per_cell;
    const int* act = d->d_active;
    double* res = d->d_results;
    void* rargs[] = {(void*)&part, (void*)&bpc, (void*)&act, (void*)&res};
    e = add((const void*)cell_reduce_kernel, dim3(d->batch), dim3(kRedThreads), rargs);
    if (e != hipSuccess) break;
    const double* resc = d->d_results;
    CellStatus* st = d->d_status;
    int* actw = d->d_active;
    int* lst = d->d_list;
    int* nact = d->d_nactive;
    int ncells = d->batch;
    double inv = 1.0 / (double)d->cell_size;
    double t = tol;
    long long ms = max_steps;
    int iv = interval;
    int pn = parity;
    void* cargs[] = {(void*)&resc, (void*)&st, (void*)&actw, (void*)&lst, (void*)&nact,
                     (void*)&ncells, (void*)&inv, (void*)&t, (void*)&ms, (void*)&iv, (void*)&pn};
    e = add((const void*)batch_check_kernel, dim3(1), dim3(1024), cargs);
  }
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(d, LBM_ERR_DEVICE, std::string("batch graph: ") + hipGetErrorString(e));
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess)
    return fail(d, LBM_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  *out = ex;
  return LBM_OK;
}

// Optional progress line on stderr (environment LBM_PROGRESS set), at most
// every 10 s, for long device-side loops.
void report_progress(lbm_domain d, int64_t steps, int running) {
  static const bool on = std::getenv("LBM_PROGRESS") != nullptr;
  if (!on) return;
  static auto last = std::chrono::steady_clock::now();
  const auto now = std::chrono::steady_clock::now();
  if (now - last < std::chrono::seconds(10)) return;
  last = now;
  std::fprintf(stderr, "[lbm] %s: %lld steps, %d running\n", d->batch ? "batch" : "domain",
               (long long)steps, running);
  std::fflush(stderr);
}

// Per-cell step parameters into the device table (relaxation rates from
// each cell's tau and Lambda, Sec. 2.1; jump from its delta_rho).
lbm_status upload_cell_params(lbm_domain d) {
  std::vector<StepParams> t(d->batch);
  for (int b = 0; b < d->batch; ++b) {
    const lbm_cell_params& c = d->cellp[b];
    StepParams& sp = t[b];
    sp.t = d->tiling;
    sp.nx = d->geo.nx;
    sp.ny = d->geo.ny;
    sp.nz = d->geo.nz_cell;
      sp.jump_axis = (1.0 / 18.0) * c.delta_rho;
    sp.jump_diag = (1.0 / 36.0) * c.delta_rho;
    sp.omega_p = 1.0 / c.tau;
    sp.omega_m = d->p.collision == LBM_TRT ? 1.0 / (0.5 + c.magic / (c.tau - 0.5)) : sp.omega_p;
    sp.s_e = 1.0 / (0.5 + (c.tau - 0.5) / 4.6);
    sp.s_zeta = 8.0 * (2.0 - sp.omega_p) / (8.0 - sp.omega_p);
    sp.sigma = 1.0;
    set_float_params(sp);
    sp.seed = 0;
    sp.wall = d->p.wall;
    sp.solid_writes = d->solid_writes;
  }
  HIP_OK(d, hipMemcpyAsync(d->d_cells, t.data(), t.size() * sizeof(StepParams),
                           hipMemcpyHostToDevice, d->stream));
  HIP_OK(d, hipStreamSynchronize(d->stream));  // t is a local host buffer
  return LBM_OK;
}

lbm_status batch_run(lbm_domain d, double tol, int64_t max_steps, int64_t* steps_done,
                     double* residual) {
  const int m = d->p.check_interval;
  const int reps = std::max(1, 512 / m);
  batch_reset_kernel<<<(d->batch + 255) / 256, 256, 0, d->stream>>>(
      d->d_status, d->d_active, d->d_list, d->d_nactive, d->batch, d->cur);
  HIP_OK(d, hipGetLastError());
  // Graphs by slot count: all cells, then the next power of two at or above
  // the running count read after each replay (the device list holds the
  // running cells, so the launch shrinks as cells stop; 256 cells of 64^3,
  // two of them run to the step limit: 71.8 -> 64.7 s for the run, whose
  // last 170k steps have few cells running).  Index: log2 of the slots (the
  // last one for all cells) and buffer parity.
  constexpr int kSlotGraphs = 32;
  hipGraphExec_t ex[kSlotGraphs][2] = {};
  lbm_status st = LBM_OK;
  int64_t done = 0;
  int nact = d->batch;
  while (done < max_steps && nact > 0) {
    int lg = 0;
    while ((1LL << lg) < nact) ++lg;
    const bool all = (1LL << lg) >= d->batch;
    const int slots = all ? d->batch : (1 << lg);
    const int gi = all ? kSlotGraphs - 1 : lg;
    hipGraphExec_t& g = ex[gi][d->cur];
    if (!g) {
      st = build_batch_graph(d, d->cur, reps, m, tol, (long long)max_steps, slots, &g);
      if (st != LBM_OK) break;
    }
    hipError_t e = hipGraphLaunch(g, d->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&nact, d->d_nactive, sizeof(int), hipMemcpyDeviceToHost, d->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
    if (e != hipSuccess) {
      st = fail(d, LBM_ERR_DEVICE, std::string("batch run: ") + hipGetErrorString(e));
      break;
    }
    const int64_t n = (int64_t)reps * m;
    done += n;
    if (n & 1) d->cur = 1 - d->cur;
    d->step_count += n;
    report_progress(d, done, nact);
  }
  for (auto& pair : ex)
    for (hipGraphExec_t g : pair)
      if (g) (void)hipGraphExecDestroy(g);
  if (st != LBM_OK) return st;
  // every cell's final state into buffer cur
  if (d->p.storage == LBM_FP64)
    batch_align_kernel<double><<<2048, 256, 0, d->stream>>>(
        (double*)d->buf[d->cur], (const double*)d->buf[1 - d->cur], d->d_status, d->cur,
        d->cell_addrs, d->tiling, d->batch);
  else
    batch_align_kernel<float><<<2048, 256, 0, d->stream>>>(
        (float*)d->buf[d->cur], (const float*)d->buf[1 - d->cur], d->d_status, d->cur,
        d->cell_addrs, d->tiling, d->batch);
  HIP_OK(d, hipGetLastError());
  d->status_host.resize(d->batch);
  HIP_OK(d, hipMemcpyAsync(d->status_host.data(), d->d_status, d->batch * sizeof(CellStatus),
                           hipMemcpyDeviceToHost, d->stream));
  HIP_OK(d, hipStreamSynchronize(d->stream));
  int64_t smax = 0;
  double rmax = 0.0;
  bool unstable = false, all_conv = true;
  for (const CellStatus& c : d->status_host) {
    smax = std::max<int64_t>(smax, c.steps);
    rmax = std::max(rmax, c.res);
    unstable |= c.status == 2;
    all_conv &= c.status == 1;
  }
  if (steps_done) *steps_done = smax;
  if (residual) *residual = rmax;
  if (unstable) {
    d->err = "at least one cell became unstable";
    return LBM_ERR_UNSTABLE;
  }
  return all_conv ? LBM_OK : LBM_ERR_NOT_CONVERGED;
}

lbm_status fetch_result(lbm_domain d, double* vals) {
  HIP_OK(d, hipGetLastError());
  HIP_OK(d, hipMemcpyAsync(vals, d->result, kRedVals * 8, hipMemcpyDeviceToHost, d->stream));
  HIP_OK(d, hipStreamSynchronize(d->stream));
  return LBM_OK;
}

// One step with the fused FP64 reduction; vals (host) after a stream sync:
// [0..2] sum u, [3] sum drho, [4] max |u|^2, [5] non-finite cells,
// [6] max_k |g_k| / w_k.
lbm_status step_and_reduce(lbm_domain d, double* vals) {
  lbm_status st = launch_step(d, true);
  if (st != LBM_OK) return st;
  const dim3 grid = step_grid(d);
  const long long nb = (long long)grid.x * grid.y * grid.z;
  const int mask = (1 << 4) | (1 << 6);
  reduce_partials_kernel<<<kRedThreads, kRedThreads, 0, d->stream>>>(d->partials, nb, mask,
                                                                     d->partials2);
  reduce_final_kernel<<<1, kRedThreads, 0, d->stream>>>(d->partials2, kRedThreads, mask,
                                                       d->result);
  return fetch_result(d, vals);
}

// Reduce the stored current state; vals as above without slot 6.  The
// kRedBlocks partial vectors go to `partials` and the final vector to
// `result` (device buffers of kRedBlocks * kRedVals and kRedVals doubles).
lbm_status reduce_state_into(lbm_domain d, double* partials, double* result, double* vals) {
  const int naddr = (int)d->naddr;
  with_storage(d->p.storage, [&](auto tag) {
    using S = decltype(tag);
    reduce_state_kernel<S><<<kRedBlocks, kRedThreads, 0, d->stream>>>(
        (const S*)d->buf[d->cur], d->flags, d->tiling, naddr, d->sigma, partials);
    return 0;
  });
  reduce_final_kernel<<<1, kRedThreads, 0, d->stream>>>(partials, kRedBlocks, 1 << 4, result);
  HIP_OK(d, hipGetLastError());
  HIP_OK(d, hipMemcpyAsync(vals, result, kRedVals * 8, hipMemcpyDeviceToHost, d->stream));
  HIP_OK(d, hipStreamSynchronize(d->stream));
  return LBM_OK;
}

// IEBB's side buffer of the current state, from its stored values (after
// the state was set from outside the time loop).
lbm_status refresh_side(lbm_domain d) {
  if (!d->side[d->cur]) return LBM_OK;
  with_storage(d->p.storage, [&](auto tag) {
    using S = decltype(tag);
    if constexpr (kUnscaledStorage<S>)
      side_moments_kernel<S><<<2048, 256, 0, d->stream>>>((const S*)d->buf[d->cur], d->cls,
                                                          d->tiling, (int)d->naddr,
                                                          d->side[d->cur]);
    return 0;
  });
  HIP_OK(d, hipGetLastError());
  return LBM_OK;
}

lbm_status reduce_state(lbm_domain d, double* vals) {
  return reduce_state_into(d, d->partials, d->result, vals);
}

// Move the 16-bit storage scale so that the largest stored magnitude
// (m * sigma) lies in [kScaleLow, kScaleHigh]; exact power-of-two rescaling
// of the current buffer.  No-op for FP32/FP64 and for BF16 (whose exponent
// range is that of FP32).
lbm_status adjust_scale(lbm_domain d, double m) {
  if (!is_fp16(d->p.storage) || !(m > 0.0) || !std::isfinite(m)) return LBM_OK;
  const double stored = m * d->sigma;
  if (stored >= kScaleLow && stored <= kScaleHigh) return LBM_OK;
  const double ns = pick_sigma(m);
  const float factor = (float)(ns / d->sigma);
  with_storage(d->p.storage, [&](auto tag) {
    using S = decltype(tag);
    rescale_kernel<S><<<2048, 256, 0, d->stream>>>((S*)d->buf[d->cur], d->flags, d->tiling,
                                                   (int)d->naddr, factor);
    return 0;
  });
  HIP_OK(d, hipGetLastError());
  d->sigma = ns;
  drop_graphs(d);
  return LBM_OK;
}

lbm_status check_ready(lbm_domain d) {
  if (!d) return LBM_ERR_INVALID_ARG;
  if (!d->bound) return fail(d, LBM_ERR_STATE, "domain is not bound to a workspace");
  return LBM_OK;
}

// Largest |g_k| / w_k of an equilibrium with the given drho and u: the
// equilibrium deviation over w is drho + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u.
double eq_magnitude(double drho, double ux, double uy, double uz) {
  const double a = std::fabs(ux) + std::fabs(uy) + std::fabs(uz);
  const double u2 = ux * ux + uy * uy + uz * uz;
  return std::fabs(drho) + 3.0 * a + 4.5 * a * a + 1.5 * u2;
}

// Scale for a new state of magnitude m (the pressure jump adds w delta_rho).
void choose_sigma(lbm_domain d, double m) {
  if (is_fp16(d->p.storage)) {
    d->sigma = pick_sigma(std::max(m, std::fabs(d->p.delta_rho)));
  } else {
    d->sigma = 1.0;
  }
  drop_graphs(d);
}

}  // namespace

// --------------------------------------------------------------- creation

LBM_API lbm_status lbm_create_domain(const uint8_t* solid_mask, const lbm_sphere* spheres,
                                     int32_t n_spheres, const lbm_params* params,
                                     lbm_domain* out) {
  g_create_error.clear();
  if (!out) return LBM_ERR_INVALID_ARG;
  *out = nullptr;
  auto bad = [](const std::string& m) {
    g_create_error = m;
    return LBM_ERR_INVALID_ARG;
  };
  if (!params) return bad("params is NULL");
  const lbm_params& p = *params;
  if (p.nx < 1 || p.ny < 1 || p.nz < 1) return bad("box edges must be >= 1");
  const int64_t ncell = (int64_t)p.nx * p.ny * p.nz;
  // the device addresses include the padding of x and y to whole tiles
  const int64_t padded = (int64_t)((p.nx + 15) / 16 * 16) * ((p.ny + 7) / 8 * 8) * p.nz;
  if (ncell >= (int64_t(1) << 31) || padded >= (int64_t(1) << 31))
    return bad("nx*ny*nz (padded to whole tiles) must be below 2^31");
  if (p.ny > 65535 || p.nz > 65535) return bad("ny and nz must be at most 65535");
  if (!(p.tau > 0.5) || !std::isfinite(p.tau)) return bad("tau must be finite and > 1/2");
  if (p.collision < LBM_SRT || p.collision > LBM_MRT) return bad("unknown collision");
  if (p.wall < LBM_WALL_SBB || p.wall > LBM_WALL_MR) return bad("unknown wall rule");
  if (p.storage < LBM_FP64 || p.storage > LBM_BF16_RNE) return bad("unknown storage");
  if (p.wall >= LBM_WALL_LIBB && p.storage != LBM_FP64 && p.storage != LBM_FP32)
    return bad("LIBB, QIBB, IEBB and MR need FP32 or FP64 storage");
  if (p.wall == LBM_WALL_IEBB && std::fabs(p.tau - 2.0) < 1e-12)
    return bad("IEBB is undefined at tau = 2 (X = (2q-1)/(tau-2))");
  if (p.collision == LBM_TRT && !(p.magic > 0.0 && p.magic <= 0.75))
    return bad("TRT magic parameter must lie in (0, 3/4]");
  if (!std::isfinite(p.delta_rho)) return bad("delta_rho must be finite");
  if (p.check_interval < 0) return bad("check_interval must be >= 0");
  const bool has_mask = solid_mask != nullptr;
  const bool has_spheres = spheres != nullptr && n_spheres > 0;
  if (n_spheres < 0) return bad("n_spheres must be >= 0");
  if (has_mask == has_spheres) return bad("give exactly one of solid_mask and spheres");
  if (has_spheres) {
    const double emin = std::min(p.nx, std::min(p.ny, p.nz));
    for (int s = 0; s < n_spheres; ++s) {
      const lbm_sphere& q = spheres[s];
      if (!(q.r > 0.0) || !(q.r < emin)) return bad("sphere radius must lie in (0, min edge)");
      if (!(q.cx >= 0 && q.cx < p.nx && q.cy >= 0 && q.cy < p.ny && q.cz >= 0 && q.cz < p.nz))
        return bad("sphere centre must lie inside the box");
    }
  }
  lbm_domain d = new (std::nothrow) lbm_domain_s();
  if (!d) return bad("out of host memory");
  d->p = p;
  if (d->p.check_interval == 0) d->p.check_interval = 100;
  std::string err;
  try {
    if (!build_geometry(solid_mask, spheres, has_spheres ? n_spheres : 0, p.nx, p.ny, p.nz,
                        d->geo, err)) {
      delete d;
      return bad(err);
    }
  } catch (const std::bad_alloc&) {
    delete d;
    return bad("out of host memory building the geometry");
  }
  // Relaxation rates (Sec. 2.1): omega+ = 1/tau = (3 nu + 1/2)^-1; TRT
  // omega- from Lambda = (1/omega+ - 1/2)(1/omega- - 1/2); MRT energy modes
  // with (1/s_nu - 1/2)/(1/s_e - 1/2) = 4.6 and Pan's s_zeta = 8(2-s_nu)/(8-s_nu).
  d->nu = (p.tau - 0.5) / 3.0;
  d->omega_p = 1.0 / p.tau;
  d->omega_m = p.collision == LBM_TRT ? 1.0 / (0.5 + p.magic / (p.tau - 0.5)) : d->omega_p;
  d->s_e = 1.0 / (0.5 + (p.tau - 0.5) / 4.6);
  d->s_zeta = 8.0 * (2.0 - d->omega_p) / (8.0 - d->omega_p);
  layout(d);
  if (d->naddr >= (int64_t(1) << 31)) {
    delete d;
    return bad("nx*ny*nz (padded to whole tiles) must be below 2^31");
  }
  if (!plane_offsets_fit(d)) {
    delete d;
    return bad("nx*ny (padded to whole tiles) must be below 2^32 / (19 * value bytes)");
  }
  choose_sigma(d, 0.0);
  *out = d;
  return LBM_OK;
}

LBM_API lbm_status lbm_get_info(lbm_domain d, lbm_info* info) {
  if (!d || !info) return LBM_ERR_INVALID_ARG;
  info->n_cells = d->geo.ncell;
  info->n_fluid = d->geo.n_fluid;
  info->n_links = (int64_t)d->geo.link_cell.size();
  info->n_fallback = d->geo.n_fallback;
  info->workspace_bytes = (int64_t)d->total;
  info->state_elems = d->state_elems;
  info->nu = d->nu;
  info->omega_plus = d->omega_p;
  info->omega_minus = d->omega_m;
  info->bytes_per_fluid_update = (int64_t)(2 * kQ * d->elem);
  info->storage_scale = d->sigma;
  info->tile_width = 1 << d->tiling.tw_log2;
  info->tile_height = 1 << d->tiling.th_log2;
  return LBM_OK;
}

LBM_API lbm_status lbm_get_mask(lbm_domain d, uint8_t* mask) {
  if (!d || !mask) return LBM_ERR_INVALID_ARG;
  std::memcpy(mask, d->geo.mask.data(), d->geo.ncell);
  return LBM_OK;
}

LBM_API lbm_status lbm_get_links(lbm_domain d, int64_t* cell, int32_t* dir, double* q,
                                 uint8_t* fallback) {
  if (!d) return LBM_ERR_INVALID_ARG;
  const size_t n = d->geo.link_cell.size();
  if (cell) std::memcpy(cell, d->geo.link_cell.data(), n * 8);
  if (dir) std::memcpy(dir, d->geo.link_dir.data(), n * 4);
  if (q) std::memcpy(q, d->geo.link_q.data(), n * 8);
  if (fallback) std::memcpy(fallback, d->geo.link_fallback.data(), n);
  return LBM_OK;
}

// ------------------------------------------------------------------ binding

LBM_API lbm_status lbm_bind(lbm_domain d, void* workspace, size_t bytes, void* stream) {
  if (!d) return LBM_ERR_INVALID_ARG;
  if (!workspace) return fail(d, LBM_ERR_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)workspace & 255) != 0)
    return fail(d, LBM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < d->total)
    return fail(d, LBM_ERR_WORKSPACE,
                "workspace too small: need " + std::to_string(d->total) + " bytes");
  d->bound = false;
  drop_graphs(d);
  {
    hipPointerAttribute_t attr{};
    HIP_OK(d, hipPointerGetAttributes(&attr, workspace));
    d->device = attr.device;
  }
  d->ws = (char*)workspace;
  d->ws_bytes = bytes;
  d->stream = (hipStream_t)stream;
  d->buf[0] = d->ws + d->off_buf[0];
  d->buf[1] = d->ws + d->off_buf[1];
  d->cur = 0;
  d->flags = (uint32_t*)(d->ws + d->off_flags);
  d->cls = (uint8_t*)(d->ws + d->off_cls);
  d->link_slot = (long long*)(d->ws + d->off_slot);
  d->link_coef = (double*)(d->ws + d->off_coef);
  d->partials = (double*)(d->ws + d->off_part);
  d->partials2 = (double*)(d->ws + d->off_part2);
  d->result = (double*)(d->ws + d->off_res);
  d->stage = (double*)(d->ws + d->off_stage);
  d->d_cells = (StepParams*)(d->ws + d->off_cells);
  d->d_active = (int*)(d->ws + d->off_active);
  d->d_active_all = (int*)(d->ws + d->off_active_all);
  d->d_status = (CellStatus*)(d->ws + d->off_status);
  d->d_results = (double*)(d->ws + d->off_results);
  d->d_nactive = (int*)(d->ws + d->off_nactive);
  d->d_list = (int*)(d->ws + d->off_list);
  for (int i = 0; i < 2; ++i) d->side[i] = d->side_bytes ? d->ws + d->off_side[i] : nullptr;
  if (d->batch) {
    lbm_status bst = upload_cell_params(d);
    if (bst != LBM_OK) return bst;
    fill_int_kernel<<<(d->batch + 255) / 256, 256, 0, d->stream>>>(d->d_active_all, d->batch, 1);
    batch_reset_kernel<<<(d->batch + 255) / 256, 256, 0, d->stream>>>(
        d->d_status, d->d_active, d->d_list, d->d_nactive, d->batch, 0);
  }

  // flag words and class bytes in tiled order (padding: solid)
  {
    const int64_t na = d->naddr;
    std::vector<uint32_t> fl((size_t)na, kSolid);
    std::vector<uint8_t> cl((size_t)na, kClsSolid);
    const int64_t cc = (int64_t)d->geo.nx * d->geo.ny * d->geo.nz_cell;
    for (int64_t c = 0; c < d->geo.ncell; ++c) {
      const int64_t b = c / cc;
      const int64_t a = b * d->cell_addrs + d->tiling.from_linear(c - b * cc);
      const uint32_t w = d->geo.flags[(size_t)c];
      fl[(size_t)a] = w;
      cl[(size_t)a] = (uint8_t)(((w & kSolid) ? kClsSolid : 0) | ((w & kLinkMask) ? kClsLinks : 0));
    }
    if (uses_side(d)) {
      // x_f2 = x + e_k of every link k at x (the link's wall is at x - e_k)
      const int nx = d->geo.nx, ny = d->geo.ny, nz = d->geo.nz;
      for (size_t i = 0; i < d->geo.link_cell.size(); ++i) {
        const int64_t c = d->geo.link_cell[i];
        const int j = d->geo.link_dir[i];  // direction from the fluid node to the wall
        const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((int64_t)nx * ny));
        const int fx = (x - kLat.ex[j] + nx) % nx, fy = (y - kLat.ey[j] + ny) % ny,
                  fz = (z - kLat.ez[j] + nz) % nz;
        const int64_t a = d->tiling.at(fx, fy, fz);
        if (!(cl[(size_t)a] & kClsSolid)) cl[(size_t)a] |= kClsNearWall;
      }
    }
    HIP_OK(d, hipMemcpyAsync(d->flags, fl.data(), (size_t)na * 4, hipMemcpyHostToDevice,
                             d->stream));
    HIP_OK(d, hipMemcpyAsync(d->cls, cl.data(), (size_t)na, hipMemcpyHostToDevice, d->stream));
    HIP_OK(d, hipStreamSynchronize(d->stream));  // fl and cl are local host buffers
  }
  // Wall-link coefficients into the slot of the solid pull source of each
  // link: link (c, j) is pulled as direction k = opp(j) from c + e_j.
  const size_t nl = d->geo.link_cell.size();
  std::vector<long long> slot(nl);
  std::vector<double> coef(nl);
  const int nx = d->geo.nx, ny = d->geo.ny;
  for (size_t i = 0; i < nl; ++i) {
    const int64_t c = d->geo.link_cell[i];
    const int j = d->geo.link_dir[i];
    const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((int64_t)nx * ny));
    // z wraps within the periodic cell (the whole box for one domain)
    const int zc = d->geo.nz_cell, z0 = z - z % zc;
    const int xs = (x + kLat.ex[j] + nx) % nx, ys = (y + kLat.ey[j] + ny) % ny,
              zs = (z - z0 + kLat.ez[j] + zc) % zc;
    const int64_t s = (int64_t)(z0 / zc) * d->cell_addrs + d->tiling.at(xs, ys, zs);
    slot[i] = d->tiling.slot(kLat.opp[j], s);
    const double q = d->geo.link_q[i];
    // eq. (CLI): a = (1 - 2q)/(1 + 2q); links without a second fluid node
    // fall back to simple bounce-back (a = 0).  The other interpolated
    // rules keep q itself and decide their fallbacks in the kernel.
    if (d->p.wall == LBM_WALL_CLI)
      coef[i] = d->geo.link_fallback[i] ? 0.0 : (1.0 - 2.0 * q) / (1.0 + 2.0 * q);
    else if (d->p.wall >= LBM_WALL_LIBB)
      coef[i] = q;
    else
      coef[i] = 0.0;
  }
  if (nl) {
    HIP_OK(d, hipMemcpyAsync(d->link_slot, slot.data(), nl * 8, hipMemcpyHostToDevice, d->stream));
    HIP_OK(d, hipMemcpyAsync(d->link_coef, coef.data(), nl * 8, hipMemcpyHostToDevice, d->stream));
  }
  const long long nel = d->state_elems;
  with_storage(d->p.storage, [&](auto tag) {
    using S = decltype(tag);
    fill_kernel<S><<<2048, 256, 0, d->stream>>>((S*)d->buf[0], nel);
    fill_kernel<S><<<2048, 256, 0, d->stream>>>((S*)d->buf[1], nel);
    if (nl)
      scatter_kernel<S><<<(int)std::min<size_t>((nl + 255) / 256, 65535), 256, 0, d->stream>>>(
          (S*)d->buf[0], (S*)d->buf[1], d->link_slot, d->link_coef, (long long)nl);
    return 0;
  });
  HIP_OK(d, hipGetLastError());
  HIP_OK(d, hipStreamSynchronize(d->stream));
  choose_sigma(d, 0.0);
  d->bound = true;
  d->unstable = false;
  return refresh_side(d);  // buffers are zero: the rest state g = 0
}

// ------------------------------------------------------------------ state

LBM_API lbm_status lbm_init_equilibrium(lbm_domain d, const double* drho0, const double* u0) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  const int64_t n = d->geo.ncell;
  double m = 0.0;
  for (int64_t c = 0; c < n; ++c) {
    if (d->geo.mask[c]) continue;
    const double r = drho0 ? drho0[c] : 0.0;
    const double ux = u0 ? u0[c] : 0.0, uy = u0 ? u0[n + c] : 0.0, uz = u0 ? u0[2 * n + c] : 0.0;
    m = std::max(m, eq_magnitude(r, ux, uy, uz));
  }
  choose_sigma(d, m);
  const size_t chunk = d->stage_cells;
  std::vector<double> host(chunk * 4);
  for (int64_t c0 = 0; c0 < n; c0 += (int64_t)chunk) {
    const int cnt = (int)std::min<int64_t>((int64_t)chunk, n - c0);
    for (int i = 0; i < cnt; ++i) {
      host[i] = drho0 ? drho0[c0 + i] : 0.0;
      host[cnt + i] = u0 ? u0[c0 + i] : 0.0;
      host[2 * cnt + i] = u0 ? u0[n + c0 + i] : 0.0;
      host[3 * cnt + i] = u0 ? u0[2 * n + c0 + i] : 0.0;
    }
    HIP_OK(d, hipMemcpyAsync(d->stage, host.data(), (size_t)cnt * 4 * 8, hipMemcpyHostToDevice,
                             d->stream));
    with_storage(d->p.storage, [&](auto tag) {
      using S = decltype(tag);
      init_eq_kernel<S><<<(cnt + 255) / 256, 256, 0, d->stream>>>(
          (S*)d->buf[d->cur], d->flags, d->tiling, cell_cells(d), (int)d->cell_addrs, d->sigma, (int)c0, cnt,
          d->stage);
      return 0;
    });
    HIP_OK(d, hipGetLastError());
    HIP_OK(d, hipStreamSynchronize(d->stream));
  }
  d->unstable = false;
  return refresh_side(d);
}

LBM_API lbm_status lbm_set_state(lbm_domain d, const double* g) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (!g) return fail(d, LBM_ERR_INVALID_ARG, "g is NULL");
  const int64_t n = d->geo.ncell;
  double m = 0.0;
  for (int k = 0; k < kQ; ++k)
    for (int64_t c = 0; c < n; ++c)
      if (!d->geo.mask[c]) m = std::max(m, std::fabs(g[(size_t)k * n + c]) / weight_of(k));
  choose_sigma(d, m);
  const size_t chunk = d->stage_cells * 4;
  for (int k = 0; k < kQ; ++k) {
    for (int64_t c0 = 0; c0 < n; c0 += (int64_t)chunk) {
      const int cnt = (int)std::min<int64_t>((int64_t)chunk, n - c0);
      HIP_OK(d, hipMemcpyAsync(d->stage, g + (size_t)k * n + c0, (size_t)cnt * 8,
                               hipMemcpyHostToDevice, d->stream));
      with_storage(d->p.storage, [&](auto tag) {
        using S = decltype(tag);
        set_plane_kernel<S><<<(cnt + 255) / 256, 256, 0, d->stream>>>(
            (S*)d->buf[d->cur], d->flags, d->tiling, cell_cells(d), (int)d->cell_addrs, k, d->sigma, (int)c0, cnt, d->stage);
        return 0;
      });
      HIP_OK(d, hipGetLastError());
      HIP_OK(d, hipStreamSynchronize(d->stream));
    }
  }
  d->unstable = false;
  return refresh_side(d);
}

LBM_API lbm_status lbm_get_state(lbm_domain d, double* g) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (!g) return fail(d, LBM_ERR_INVALID_ARG, "g is NULL");
  const int64_t n = d->geo.ncell;
  const size_t chunk = d->stage_cells * 4;
  for (int k = 0; k < kQ; ++k) {
    for (int64_t c0 = 0; c0 < n; c0 += (int64_t)chunk) {
      const int cnt = (int)std::min<int64_t>((int64_t)chunk, n - c0);
      with_storage(d->p.storage, [&](auto tag) {
        using S = decltype(tag);
        get_plane_kernel<S><<<(cnt + 255) / 256, 256, 0, d->stream>>>(
            (const S*)d->buf[d->cur], d->flags, d->tiling, cell_cells(d), (int)d->cell_addrs, k, d->sigma, (int)c0, cnt, d->stage);
        return 0;
      });
      HIP_OK(d, hipGetLastError());
      HIP_OK(d, hipMemcpyAsync(g + (size_t)k * n + c0, d->stage, (size_t)cnt * 8,
                               hipMemcpyDeviceToHost, d->stream));
      HIP_OK(d, hipStreamSynchronize(d->stream));
    }
  }
  return LBM_OK;
}

// ------------------------------------------------------------------ stepping

LBM_API lbm_status lbm_step(lbm_domain d, int64_t n) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (n < 0) return fail(d, LBM_ERR_INVALID_ARG, "n must be >= 0");
  if (d->unstable) return fail(d, LBM_ERR_STATE, "state is unstable; re-initialise first");
  return d->batch ? enqueue_batch_steps(d, n) : enqueue_steps(d, n);
}

LBM_API lbm_status lbm_run_to_residual(lbm_domain d, double tol, int64_t max_steps,
                                       int64_t* steps_done, double* residual) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (max_steps < 0 || !(tol >= 0)) return fail(d, LBM_ERR_INVALID_ARG, "bad tol or max_steps");
  if (d->unstable) return fail(d, LBM_ERR_STATE, "state is unstable; re-initialise first");
  if (d->batch) return batch_run(d, tol, max_steps, steps_done, residual);
  const double cs2 = 1.0 / 3.0;
  const double ncell = (double)d->geo.ncell;
  double v[kRedVals];
  st = reduce_state(d, v);
  if (st != LBM_OK) return st;
  double prev = v[0] / ncell, res = INFINITY;
  int64_t done = 0;
  int below = 0;
  lbm_status out = LBM_ERR_NOT_CONVERGED;
  while (done < max_steps) {
    const int64_t m = std::min<int64_t>(d->p.check_interval, max_steps - done);
    st = enqueue_steps(d, m - 1);
    if (st != LBM_OK) return st;
    st = step_and_reduce(d, v);  // the m-th step also reduces the new state
    if (st != LBM_OK) return st;
    done += m;
    const double U = v[0] / ncell;
    if (v[5] > 0 || !std::isfinite(U) || v[4] > cs2) {
      d->unstable = true;
      out = LBM_ERR_UNSTABLE;
      d->err = "non-finite state or |u| above the sound speed";
      break;
    }
    st = adjust_scale(d, v[6]);
    if (st != LBM_OK) return st;
    res = U != 0.0 ? std::fabs(U - prev) / std::fabs(U) : (U == prev ? 0.0 : INFINITY);
    prev = U;
    below = res < tol ? below + 1 : 0;
    if (below >= 3) {
      out = LBM_OK;
      break;
    }
    report_progress(d, done, 1);
  }
  if (steps_done) *steps_done = done;
  if (residual) *residual = res;
  return out;
}

// --------------------------------------------------------------- observables

LBM_API lbm_status lbm_macroscopic(lbm_domain d, double* drho, double* u) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  const int64_t n = d->geo.ncell;
  const size_t chunk = d->stage_cells;
  std::vector<double> host(chunk * 4);
  for (int64_t c0 = 0; c0 < n; c0 += (int64_t)chunk) {
    const int cnt = (int)std::min<int64_t>((int64_t)chunk, n - c0);
    with_storage(d->p.storage, [&](auto tag) {
      using S = decltype(tag);
      macro_kernel<S><<<(cnt + 255) / 256, 256, 0, d->stream>>>(
          (const S*)d->buf[d->cur], d->flags, d->tiling, cell_cells(d), (int)d->cell_addrs, d->sigma, (int)c0, cnt,
          d->stage);
      return 0;
    });
    HIP_OK(d, hipGetLastError());
    HIP_OK(d, hipMemcpyAsync(host.data(), d->stage, (size_t)cnt * 4 * 8, hipMemcpyDeviceToHost,
                             d->stream));
    HIP_OK(d, hipStreamSynchronize(d->stream));
    for (int i = 0; i < cnt; ++i) {
      if (drho) drho[c0 + i] = host[i];
      if (u) {
        u[c0 + i] = host[cnt + i];
        u[n + c0 + i] = host[2 * cnt + i];
        u[2 * n + c0 + i] = host[3 * cnt + i];
      }
    }
  }
  return LBM_OK;
}

LBM_API lbm_status lbm_macroscopic_device(lbm_domain d, double* fields) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (!fields) return fail(d, LBM_ERR_INVALID_ARG, "fields is NULL");
  const int n = (int)d->geo.ncell;
  with_storage(d->p.storage, [&](auto tag) {
    using S = decltype(tag);
    macro_kernel<S><<<(n + 255) / 256, 256, 0, d->stream>>>(
        (const S*)d->buf[d->cur], d->flags, d->tiling, cell_cells(d), (int)d->cell_addrs, d->sigma, 0, n, fields);
    return 0;
  });
  HIP_OK(d, hipGetLastError());
  return LBM_OK;
}

LBM_API lbm_status lbm_init_equilibrium_device(lbm_domain d, const double* fields) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (!fields) return fail(d, LBM_ERR_INVALID_ARG, "fields is NULL");
  if (d->p.storage != LBM_FP32 && d->p.storage != LBM_FP64)
    return fail(d, LBM_ERR_INVALID_ARG,
                "device initialisation needs FP32 or FP64 storage (16-bit storage chooses its "
                "scale from the host fields)");
  const int n = (int)d->geo.ncell;
  with_storage(d->p.storage, [&](auto tag) {
    using S = decltype(tag);
    init_eq_kernel<S><<<(n + 255) / 256, 256, 0, d->stream>>>(
        (S*)d->buf[d->cur], d->flags, d->tiling, cell_cells(d), (int)d->cell_addrs, d->sigma, 0, n, fields);
    return 0;
  });
  HIP_OK(d, hipGetLastError());
  d->unstable = false;
  return refresh_side(d);
}

// Outputs of lbm_mean_velocity from the reduced vector.
static void mean_velocity_outputs(lbm_domain d, const double* v, double U[3], double* max_speed,
                           double* total_drho) {
  const double n = (double)d->geo.ncell;
  if (U) {
    U[0] = v[0] / n;
    U[1] = v[1] / n;
    U[2] = v[2] / n;
  }
  if (max_speed) *max_speed = v[5] > 0 ? NAN : std::sqrt(v[4]);
  if (total_drho) *total_drho = v[3];
}

LBM_API lbm_status lbm_mean_velocity(lbm_domain d, double U[3], double* max_speed,
                                     double* total_drho) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (d->batch) return fail(d, LBM_ERR_STATE, "per-domain call on a batch; use lbm_batch_results");
  double v[kRedVals];
  st = reduce_state(d, v);
  if (st != LBM_OK) return st;
  mean_velocity_outputs(d, v, U, max_speed, total_drho);
  return LBM_OK;
}

// ------------------------------------------------- no-allocation variant
// Scratch of lbm_mean_velocity_static: the block partial sums and the final
// vector of the state reduction live in this device array of the library
// (one copy per GPU, held until the process ends) instead of the domain's
// workspace.  Host code never passes the array's name to a kernel or a copy:
// it uses the device address that hipGetSymbolAddress returns for the GPU in
// question (kept per device below).
constexpr int kStaticPartials = kRedBlocks;  // the state reduction's fixed grid
constexpr int kStaticScratchDoubles = kStaticPartials * kRedVals + kRedVals;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the domain's GPU, looked up once per device
// with that device current (the caller's current device is restored).
lbm_status static_scratch(lbm_domain d, double** out) {
  if (d->device < 0 || d->device >= kMaxDevices)
    return fail(d, LBM_ERR_DEVICE, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[d->device]) {
    int prev = 0;
    HIP_OK(d, hipGetDevice(&prev));
    if (prev != d->device) HIP_OK(d, hipSetDevice(d->device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != d->device) HIP_OK(d, hipSetDevice(prev));
    if (e != hipSuccess || !p)
      return fail(d, LBM_ERR_DEVICE,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[d->device] = (double*)p;
  }
  *out = g_scratch_ptr[d->device];
  return LBM_OK;
}
}  // namespace

LBM_API lbm_status lbm_mean_velocity_static(lbm_domain d, double U[3], double* max_speed,
                                            double* total_drho) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (d->batch) return fail(d, LBM_ERR_STATE, "per-domain call on a batch; use lbm_batch_results");
  // the reduction runs a fixed grid of kRedBlocks blocks whatever the domain
  // size, so its scratch never exceeds the array; checked all the same
  if ((long long)kRedBlocks * kRedVals + kRedVals > kStaticScratchDoubles)
    return fail(d, LBM_ERR_INVALID_ARG, "reduction needs more scratch than the static array holds");
  double* scr = nullptr;
  st = static_scratch(d, &scr);
  if (st != LBM_OK) return st;
  double v[kRedVals];
  st = reduce_state_into(d, scr, scr + kStaticPartials * kRedVals, v);
  if (st != LBM_OK) return st;
  mean_velocity_outputs(d, v, U, max_speed, total_drho);
  return LBM_OK;
}

// eq. (Darcy): K_D = mu U / |grad P| with mu = nu (rho0 = 1), |grad P| = dp/nx,
// dp = delta_rho / 3; Re_p / D = U / nu (Sec. 1, rho = 1).
LBM_API lbm_status lbm_permeability(lbm_domain d, double* K_D, double* U_x,
                                    double* Re_p_per_D) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (d->batch) return fail(d, LBM_ERR_STATE, "per-domain call on a batch; use lbm_batch_results");
  if (d->p.delta_rho == 0.0) return fail(d, LBM_ERR_STATE, "delta_rho is zero");
  double U[3];
  st = lbm_mean_velocity(d, U, nullptr, nullptr);
  if (st != LBM_OK) return st;
  const double dp = d->p.delta_rho / 3.0;
  if (K_D) *K_D = d->nu * U[0] * d->geo.nx / dp;
  if (U_x) *U_x = U[0];
  if (Re_p_per_D) *Re_p_per_D = U[0] / d->nu;
  return LBM_OK;
}

LBM_API lbm_status lbm_drag(lbm_domain d, double F[3]) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (d->batch) return fail(d, LBM_ERR_STATE, "per-domain call on a batch; use lbm_batch_results");
  if (!F) return fail(d, LBM_ERR_INVALID_ARG, "F is NULL");
  StepParams sp = step_params(d);
  // the drag kernel computes in FP64 and sums IEBB's x_f2 values itself
  sp.side_in = sp.side_out = nullptr;
  const bool cli = d->p.wall == LBM_WALL_CLI;
  const bool gen = wall_template(d->p.wall) == kGEN;
  with_storage(d->p.storage, [&](auto tag) {
    using S = decltype(tag);
    if constexpr (kUnscaledStorage<S>) {
      if (gen) {
        drag_kernel<S, kGEN><<<kRedBlocks, kRedThreads, 0, d->stream>>>(
            (const S*)d->buf[d->cur], d->flags, sp, d->partials);
        return 0;
      }
    }
    if (cli)
      drag_kernel<S, kCLI><<<kRedBlocks, kRedThreads, 0, d->stream>>>(
          (const S*)d->buf[d->cur], d->flags, sp, d->partials);
    else
      drag_kernel<S, kSBB><<<kRedBlocks, kRedThreads, 0, d->stream>>>(
          (const S*)d->buf[d->cur], d->flags, sp, d->partials);
    return 0;
  });
  reduce_final_kernel<<<1, kRedThreads, 0, d->stream>>>(d->partials, kRedBlocks, 0, d->result);
  double v[kRedVals];
  st = fetch_result(d, v);
  if (st != LBM_OK) return st;
  F[0] = v[0];
  F[1] = v[1];
  F[2] = v[2];
  return LBM_OK;
}

// ------------------------------------------------------------------ batches

LBM_API lbm_status lbm_create_batch(int32_t n_cells, const uint8_t* masks,
                                    const lbm_sphere* spheres, const int32_t* sphere_counts,
                                    const lbm_cell_params* cells, const lbm_params* common,
                                    lbm_domain* out) {
  g_create_error.clear();
  if (!out) return LBM_ERR_INVALID_ARG;
  *out = nullptr;
  auto bad = [](const std::string& m) {
    g_create_error = m;
    return LBM_ERR_INVALID_ARG;
  };
  if (n_cells < 1 || !cells || !common) return bad("n_cells >= 1, cells and common are required");
  const lbm_params& p = *common;
  if (p.nx < 1 || p.ny < 1 || p.nz < 1) return bad("box edges must be >= 1");
  const int64_t csize = (int64_t)p.nx * p.ny * p.nz;
  if (csize * n_cells >= (int64_t(1) << 31)) return bad("n_cells*nx*ny*nz must be below 2^31");
  if (p.ny > 65535 || (int64_t)p.nz * n_cells > 65535 * 64)
    return bad("ny must be at most 65535 and n_cells*nz at most 65535*64");
  if (p.collision < LBM_SRT || p.collision > LBM_MRT) return bad("unknown collision");
  if (p.wall < LBM_WALL_SBB || p.wall > LBM_WALL_MR) return bad("unknown wall rule");
  if (p.storage != LBM_FP64 && p.storage != LBM_FP32) return bad("batches store FP32 or FP64");
  if (p.check_interval < 0) return bad("check_interval must be >= 0");
  if ((masks != nullptr) == (spheres != nullptr)) return bad("give exactly one of masks and spheres");
  if (spheres && !sphere_counts) return bad("sphere_counts is required with spheres");
  for (int b = 0; b < n_cells; ++b) {
    const lbm_cell_params& c = cells[b];
    if (!(c.tau > 0.5) || !std::isfinite(c.tau)) return bad("cell tau must be finite and > 1/2");
    if (p.wall == LBM_WALL_IEBB && std::fabs(c.tau - 2.0) < 1e-12)
      return bad("IEBB is undefined at tau = 2 (X = (2q-1)/(tau-2))");
    if (p.collision == LBM_TRT && !(c.magic > 0.0 && c.magic <= 0.75))
      return bad("cell TRT magic parameter must lie in (0, 3/4]");
    if (!std::isfinite(c.delta_rho)) return bad("cell delta_rho must be finite");
  }
  const double emin = std::min(p.nx, std::min(p.ny, p.nz));
  if (spheres) {
    int64_t at = 0;
    for (int b = 0; b < n_cells; ++b) {
      if (sphere_counts[b] < 1) return bad("every cell needs at least one sphere");
      for (int i = 0; i < sphere_counts[b]; ++i) {
        const lbm_sphere& q = spheres[at + i];
        if (!(q.r > 0.0) || !(q.r < emin)) return bad("sphere radius must lie in (0, min edge)");
        if (!(q.cx >= 0 && q.cx < p.nx && q.cy >= 0 && q.cy < p.ny && q.cz >= 0 && q.cz < p.nz))
          return bad("sphere centre must lie inside the cell");
      }
      at += sphere_counts[b];
    }
  }
  lbm_domain d = new (std::nothrow) lbm_domain_s();
  if (!d) return bad("out of host memory");
  d->p = p;
  if (d->p.check_interval == 0) d->p.check_interval = 100;
  d->batch = n_cells;
  d->cell_size = csize;
  d->cellp.assign(cells, cells + n_cells);
  try {
    int64_t at = 0;
    for (int b = 0; b < n_cells; ++b) {
      Geometry g;
      std::string err;
      const uint8_t* m = masks ? masks + (size_t)b * csize : nullptr;
      const lbm_sphere* sp = spheres ? spheres + at : nullptr;
      const int ns = spheres ? sphere_counts[b] : 0;
      if (spheres) at += sphere_counts[b];
      if (!build_geometry(m, sp, ns, p.nx, p.ny, p.nz, g, err)) {
        delete d;
        return bad("cell " + std::to_string(b) + ": " + err);
      }
      append_cell(d->geo, g);
    }
  } catch (const std::bad_alloc&) {
    delete d;
    return bad("out of host memory building the geometry");
  }
  d->nu = (cells[0].tau - 0.5) / 3.0;
  d->omega_p = 1.0 / cells[0].tau;
  d->omega_m = d->omega_p;
  d->bby = 4;  // wavefronts (tiles) per workgroup until set or autotuned
  d->zper = 1;
  layout(d);
  if (d->naddr >= (int64_t(1) << 31)) {
    delete d;
    return bad("n_cells*nx*ny*nz (padded to whole tiles) must be below 2^31");
  }
  if (!plane_offsets_fit(d)) {
    delete d;
    return bad("nx*ny (padded to whole tiles) must be below 2^32 / (19 * value bytes)");
  }
  choose_sigma(d, 0.0);
  *out = d;
  return LBM_OK;
}

LBM_API lbm_status lbm_batch_results(lbm_domain d, double* U, double* K_D, int64_t* steps,
                                     double* residual, int32_t* status) {
  if (!d || !d->batch) return LBM_ERR_INVALID_ARG;
  if (d->status_host.size() != (size_t)d->batch)
    return fail(d, LBM_ERR_STATE, "no residual run on this batch yet");
  for (int b = 0; b < d->batch; ++b) {
    const CellStatus& c = d->status_host[b];
    if (U) {
      U[3 * b] = c.u[0];
      U[3 * b + 1] = c.u[1];
      U[3 * b + 2] = c.u[2];
    }
    if (K_D) {
      const lbm_cell_params& cp = d->cellp[b];
      const double nu = (cp.tau - 0.5) / 3.0;
      K_D[b] = cp.delta_rho != 0.0 ? nu * c.u[0] * d->geo.nx / (cp.delta_rho / 3.0) : NAN;
    }
    if (steps) steps[b] = c.steps;
    if (residual) residual[b] = c.res;
    if (status) status[b] = c.status;
  }
  return LBM_OK;
}

LBM_API lbm_status lbm_set_step_shape(lbm_domain d, int32_t waves, int32_t rows,
                                      int32_t pairs) {
  if (!d || d->batch) return LBM_ERR_INVALID_ARG;
  if (waves != 1 && waves != 2 && waves != 4 && waves != 8 && waves != 16)
    return fail(d, LBM_ERR_INVALID_ARG, "waves must be 1, 2, 4, 8 or 16");
  if (rows < 1 || waves % rows != 0)
    return fail(d, LBM_ERR_INVALID_ARG, "rows must divide waves");
  if (pairs != 0 && pairs != 1) return fail(d, LBM_ERR_INVALID_ARG, "pairs must be 0 or 1");
  if (pairs && (d->elem != 2 || d->geo.nx % (1 << d->tiling.tw_log2) != 0))
    return fail(d, LBM_ERR_INVALID_ARG,
                "two cells per lane need 16-bit storage and nx a multiple of the tile width " +
                    std::to_string(1 << d->tiling.tw_log2));
  const int old_waves = d->waves, old_rows = d->rows;
  const bool old_pairs = d->pairs;
  d->waves = waves;
  d->rows = rows;
  d->pairs = pairs != 0;
  const dim3 g = step_grid(d);
  if ((long long)g.x * g.y * g.z > d->n_partials) {
    d->waves = old_waves;
    d->rows = old_rows;
    d->pairs = old_pairs;
    return fail(d, LBM_ERR_INVALID_ARG, "shape needs more partial sums than the workspace holds");
  }
  drop_graphs(d);
  return LBM_OK;
}

LBM_API lbm_status lbm_get_step_shape(lbm_domain d, int32_t* waves, int32_t* rows,
                                      int32_t* pairs) {
  if (!d || d->batch) return LBM_ERR_INVALID_ARG;
  if (waves) *waves = d->waves;
  if (rows) *rows = d->rows;
  if (pairs) *pairs = d->pairs ? 1 : 0;
  return LBM_OK;
}

LBM_API lbm_status lbm_batch_set_shape(lbm_domain d, int32_t waves, int32_t zper) {
  if (!d || !d->batch) return LBM_ERR_INVALID_ARG;
  if (waves < 1 || 64 * waves > kBatchThreads || zper < 1 || d->geo.nz_cell % zper != 0)
    return fail(d, LBM_ERR_INVALID_ARG,
                "waves must lie in [1, " + std::to_string(kBatchThreads / 64) +
                    "] and zper must divide nz");
  d->bby = waves;
  d->zper = zper;
  return LBM_OK;
}

// Rest state again after tuning: zero both buffers, re-scatter coefficients.
static lbm_status reset_to_rest(lbm_domain d) {
  void* ws = d->ws;
  size_t bytes = d->ws_bytes;
  hipStream_t stream = d->stream;
  const int by = d->bby, zp = d->zper;
  lbm_status st = lbm_bind(d, ws, bytes, stream);
  d->bby = by;
  d->zper = zp;
  return st;
}

LBM_API lbm_status lbm_batch_autotune(lbm_domain d, int32_t steps, int32_t* by_out,
                                      int32_t* zper_out, double* ms_out) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (!d->batch) return fail(d, LBM_ERR_STATE, "autotune applies to batches");
  if (steps < 1) return fail(d, LBM_ERR_INVALID_ARG, "steps must be >= 1");
  const int tiles = d->tiling.ntx * d->tiling.nty;
  hipEvent_t e0, e1;
  HIP_OK(d, hipEventCreate(&e0));
  HIP_OK(d, hipEventCreate(&e1));
  double best = INFINITY;
  int best_by = d->bby, best_z = d->zper, best_mode = d->solid_writes;
  for (int mode = 0; mode <= 2 && st == LBM_OK; ++mode) {
    d->solid_writes = mode;
    st = upload_cell_params(d);
    if (st != LBM_OK) break;
    for (int by = 1; 64 * by <= kBatchThreads && by <= tiles; by *= 2) {
      for (int zp = 1; zp <= 8 && zp <= d->geo.nz_cell; zp *= 2) {
        if (d->geo.nz_cell % zp) continue;
        d->bby = by;
        d->zper = zp;
        st = enqueue_batch_steps(d, 2);
        if (st != LBM_OK) break;
        HIP_OK(d, hipEventRecord(e0, d->stream));
        st = enqueue_batch_steps(d, steps);
        if (st != LBM_OK) break;
        HIP_OK(d, hipEventRecord(e1, d->stream));
        HIP_OK(d, hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_OK(d, hipEventElapsedTime(&ms, e0, e1));
        const double per = ms / steps;
        if (per < best) {
          best = per;
          best_by = by;
          best_z = zp;
          best_mode = mode;
        }
      }
      if (st != LBM_OK) break;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  d->solid_writes = best_mode;
  if (st != LBM_OK) return st;
  d->bby = best_by;
  d->zper = best_z;
  st = reset_to_rest(d);
  if (st != LBM_OK) return st;
  if (by_out) *by_out = best_by;
  if (zper_out) *zper_out = best_z;
  if (ms_out) *ms_out = best;
  return LBM_OK;
}

LBM_API lbm_status lbm_set_solid_writes(lbm_domain d, int32_t mode) {
  if (!d) return LBM_ERR_INVALID_ARG;
  if (mode < 0 || mode > 2) return fail(d, LBM_ERR_INVALID_ARG, "solid_writes must be 0, 1 or 2");
  if (!d->batch && mode != 0) return fail(d, LBM_ERR_STATE, "solid writes apply to batches");
  d->solid_writes = mode;
  if (d->batch && d->ws) return upload_cell_params(d);
  return LBM_OK;
}

LBM_API lbm_status lbm_get_solid_writes(lbm_domain d, int32_t* mode) {
  if (!d || !mode) return LBM_ERR_INVALID_ARG;
  *mode = d->solid_writes;
  return LBM_OK;
}

LBM_API lbm_status lbm_set_delta_rho(lbm_domain d, double delta_rho) {
  if (!d) return LBM_ERR_INVALID_ARG;
  if (d->batch) return fail(d, LBM_ERR_STATE, "per-domain call on a batch");
  if (!std::isfinite(delta_rho)) return fail(d, LBM_ERR_INVALID_ARG, "delta_rho must be finite");
  d->p.delta_rho = delta_rho;
  drop_graphs(d);
  return LBM_OK;
}

LBM_API lbm_status lbm_synchronize(lbm_domain d) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  HIP_OK(d, hipStreamSynchronize(d->stream));
  return LBM_OK;
}

LBM_API lbm_status lbm_destroy(lbm_domain d) {
  if (!d) return LBM_ERR_INVALID_ARG;
  if (d->bound) (void)hipStreamSynchronize(d->stream);
  drop_graphs(d);
  delete d;
  return LBM_OK;
}

LBM_API const char* lbm_status_string(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_ERR_INVALID_ARG: return "invalid argument";
    case LBM_ERR_WORKSPACE: return "workspace missing or too small";
    case LBM_ERR_DEVICE: return "device error";
    case LBM_ERR_UNSTABLE: return "unstable state";
    case LBM_ERR_NOT_CONVERGED: return "not converged";
    case LBM_ERR_STATE: return "invalid state for this call";
  }
  return "unknown status";
}

LBM_API const char* lbm_last_error(lbm_domain d) {
  return d ? d->err.c_str() : g_create_error.c_str();
}
