// C ABI of the D3Q19 hot path (include/lbm.h): domain lifetime, workspace
// layout, kernel launches and host-side control of the time loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "geometry.hpp"
#include "kernels.hpp"
#include "lbm.h"

#define LBM_API extern "C" __attribute__((visibility("default")))

using namespace lbm;

struct lbm_domain_s {
  lbm_params p{};
  Geometry geo;
  std::string err;
  // derived
  long long stride = 0;  // elements per direction plane
  size_t elem = 0;       // bytes per stored population
  double nu = 0, omega_p = 0, omega_m = 0, s_e = 0, s_zeta = 0;
  double sigma = 1.0;    // 16-bit storage scale (h = sigma g / w), a power of two
  uint64_t step_count = 0;  // steps launched (seeds stochastic rounding)
  // device (inside the caller's workspace)
  bool bound = false;
  bool unstable = false;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  void* buf[2] = {nullptr, nullptr};
  int cur = 0;  // buf[cur] holds the current state
  uint32_t* flags = nullptr;
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
  // layout offsets
  size_t off_buf[2] = {0, 0}, off_flags = 0, off_slot = 0, off_coef = 0, off_part = 0,
         off_part2 = 0, off_res = 0, off_stage = 0, total = 0;
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

// Direction planes are padded so that the 19 streams do not start on the same
// HBM channel: round the cell count up to 1024 elements, plus 512 elements.
long long plane_stride(int64_t ncell) { return (long long)(((ncell + 1023) / 1024) * 1024 + 512); }

// Workgroups cover full x rows (up to 512 cells) and 256/bx rows in y.
dim3 step_block(int nx) {
  const int bx = std::min(512, ((nx + 63) / 64) * 64);
  const int by = std::max(1, 256 / bx);
  return dim3(bx, by, 1);
}
dim3 step_grid(int nx, int ny, int nz) {
  const dim3 b = step_block(nx);
  return dim3((nx + b.x - 1) / b.x, (ny + b.y - 1) / b.y, nz);
}

void layout(lbm_domain d) {
  const int64_t n = d->geo.ncell;
  d->stride = plane_stride(n);
  d->elem = storage_bytes(d->p.storage);
  size_t o = 0;
  const size_t bufb = align256((size_t)kQ * d->stride * d->elem);
  d->off_buf[0] = o;
  o += bufb;
  d->off_buf[1] = o;
  o += bufb;
  d->off_flags = o;
  o += align256((size_t)n * 4);
  const size_t nl = d->geo.link_cell.size();
  d->off_slot = o;
  o += align256(std::max<size_t>(nl, 1) * 8);
  d->off_coef = o;
  o += align256(std::max<size_t>(nl, 1) * 8);
  const dim3 sg = step_grid(d->geo.nx, d->geo.ny, d->geo.nz);
  d->n_partials = std::max<long long>(kRedBlocks, (long long)sg.x * sg.y * sg.z);
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
  d->total = o;
}

StepParams step_params(lbm_domain d) {
  StepParams sp;
  sp.nx = d->geo.nx;
  sp.ny = d->geo.ny;
  sp.nz = d->geo.nz;
  sp.stride = d->stride;
  sp.jump_axis = (1.0 / 18.0) * d->p.delta_rho;
  sp.jump_diag = (1.0 / 36.0) * d->p.delta_rho;
  sp.omega_p = d->omega_p;
  sp.omega_m = d->omega_m;
  sp.s_e = d->s_e;
  sp.s_zeta = d->s_zeta;
  sp.sigma = d->sigma;
  sp.seed = hash32((uint32_t)d->step_count ^ hash32((uint32_t)(d->step_count >> 32) + 0x5bd1e995u));
  return sp;
}

template <typename S, bool RED>
const void* step_fn(int collision, int wall) {
  switch (collision * 2 + wall) {
    case 0: return (const void*)step_kernel<S, kSRT, kSBB, RED>;
    case 1: return (const void*)step_kernel<S, kSRT, kCLI, RED>;
    case 2: return (const void*)step_kernel<S, kTRT, kSBB, RED>;
    case 3: return (const void*)step_kernel<S, kTRT, kCLI, RED>;
    case 4: return (const void*)step_kernel<S, kMRT, kSBB, RED>;
    default: return (const void*)step_kernel<S, kMRT, kCLI, RED>;
  }
}

const void* step_function(lbm_domain d, bool red) {
  return with_storage(d->p.storage, [&](auto tag) -> const void* {
    using S = decltype(tag);
    return red ? step_fn<S, true>(d->p.collision, d->p.wall)
               : step_fn<S, false>(d->p.collision, d->p.wall);
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
  uint32_t* fl = d->flags;
  double* part = d->partials;
  void* args[] = {(void*)&src, (void*)&dst, (void*)&fl, (void*)&sp, (void*)&part};
  const dim3 grid = step_grid(d->geo.nx, d->geo.ny, d->geo.nz), block = step_block(d->geo.nx);
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
  uint32_t* fl = d->flags;
  double* part = d->partials;
  const dim3 grid = step_grid(d->geo.nx, d->geo.ny, d->geo.nz), block = step_block(d->geo.nx);
  const void* fn = step_function(d, false);
  hipGraphNode_t prev = nullptr;
  for (int i = 0; i < kGraphSteps; ++i) {
    const void* src = d->buf[(from + i) & 1];
    void* dst = d->buf[(from + i + 1) & 1];
    void* args[] = {(void*)&src, (void*)&dst, (void*)&fl, (void*)&sp, (void*)&part};
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
  const dim3 grid = step_grid(d->geo.nx, d->geo.ny, d->geo.nz);
  const long long nb = (long long)grid.x * grid.y * grid.z;
  const int mask = (1 << 4) | (1 << 6);
  reduce_partials_kernel<<<kRedThreads, kRedThreads, 0, d->stream>>>(d->partials, nb, mask,
                                                                     d->partials2);
  reduce_final_kernel<<<1, kRedThreads, 0, d->stream>>>(d->partials2, kRedThreads, mask,
                                                       d->result);
  return fetch_result(d, vals);
}

// Reduce the stored current state; vals as above without slot 6.
lbm_status reduce_state(lbm_domain d, double* vals) {
  const int ncell = (int)d->geo.ncell;
  with_storage(d->p.storage, [&](auto tag) {
    using S = decltype(tag);
    reduce_state_kernel<S><<<kRedBlocks, kRedThreads, 0, d->stream>>>(
        (const S*)d->buf[d->cur], d->flags, d->stride, ncell, d->sigma, d->partials);
    return 0;
  });
  reduce_final_kernel<<<1, kRedThreads, 0, d->stream>>>(d->partials, kRedBlocks, 1 << 4,
                                                       d->result);
  return fetch_result(d, vals);
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
    rescale_kernel<S><<<2048, 256, 0, d->stream>>>((S*)d->buf[d->cur], d->flags, d->stride,
                                                   (int)d->geo.ncell, factor);
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
  if (ncell >= (int64_t(1) << 31)) return bad("nx*ny*nz must be below 2^31");
  if (p.ny > 65535 || p.nz > 65535) return bad("ny and nz must be at most 65535");
  if (!(p.tau > 0.5) || !std::isfinite(p.tau)) return bad("tau must be finite and > 1/2");
  if (p.collision < LBM_SRT || p.collision > LBM_MRT) return bad("unknown collision");
  if (p.wall < LBM_WALL_SBB || p.wall > LBM_WALL_CLI) return bad("unknown wall rule");
  if (p.storage < LBM_FP64 || p.storage > LBM_BF16_RNE) return bad("unknown storage");
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
  info->plane_stride = d->stride;
  info->nu = d->nu;
  info->omega_plus = d->omega_p;
  info->omega_minus = d->omega_m;
  info->bytes_per_fluid_update = (int64_t)(2 * kQ * d->elem);
  info->storage_scale = d->sigma;
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
  d->ws = (char*)workspace;
  d->ws_bytes = bytes;
  d->stream = (hipStream_t)stream;
  d->buf[0] = d->ws + d->off_buf[0];
  d->buf[1] = d->ws + d->off_buf[1];
  d->cur = 0;
  d->flags = (uint32_t*)(d->ws + d->off_flags);
  d->link_slot = (long long*)(d->ws + d->off_slot);
  d->link_coef = (double*)(d->ws + d->off_coef);
  d->partials = (double*)(d->ws + d->off_part);
  d->partials2 = (double*)(d->ws + d->off_part2);
  d->result = (double*)(d->ws + d->off_res);
  d->stage = (double*)(d->ws + d->off_stage);

  const int64_t n = d->geo.ncell;
  HIP_OK(d, hipMemcpyAsync(d->flags, d->geo.flags.data(), n * 4, hipMemcpyHostToDevice,
                           d->stream));
  // Wall-link coefficients into the slot of the solid pull source of each
  // link: link (c, j) is pulled as direction k = opp(j) from c + e_j.
  const size_t nl = d->geo.link_cell.size();
  std::vector<long long> slot(nl);
  std::vector<double> coef(nl);
  const int nx = d->geo.nx, ny = d->geo.ny, nz = d->geo.nz;
  for (size_t i = 0; i < nl; ++i) {
    const int64_t c = d->geo.link_cell[i];
    const int j = d->geo.link_dir[i];
    const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((int64_t)nx * ny));
    const int xs = (x + kLat.ex[j] + nx) % nx, ys = (y + kLat.ey[j] + ny) % ny,
              zs = (z + kLat.ez[j] + nz) % nz;
    const int64_t s = xs + (int64_t)nx * (ys + (int64_t)ny * zs);
    slot[i] = (long long)kLat.opp[j] * d->stride + s;
    const double q = d->geo.link_q[i];
    // eq. (CLI): a = (1 - 2q)/(1 + 2q); links without a second fluid node
    // fall back to simple bounce-back (a = 0)
    coef[i] = (d->p.wall == LBM_WALL_CLI && !d->geo.link_fallback[i])
                  ? (1.0 - 2.0 * q) / (1.0 + 2.0 * q)
                  : 0.0;
  }
  if (nl) {
    HIP_OK(d, hipMemcpyAsync(d->link_slot, slot.data(), nl * 8, hipMemcpyHostToDevice, d->stream));
    HIP_OK(d, hipMemcpyAsync(d->link_coef, coef.data(), nl * 8, hipMemcpyHostToDevice, d->stream));
  }
  const long long nel = (long long)kQ * d->stride;
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
  return LBM_OK;  // buffers are zero: the rest state g = 0
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
          (S*)d->buf[d->cur], d->flags, d->stride, d->sigma, (int)c0, cnt, d->stage);
      return 0;
    });
    HIP_OK(d, hipGetLastError());
    HIP_OK(d, hipStreamSynchronize(d->stream));
  }
  d->unstable = false;
  return LBM_OK;
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
    char* plane = (char*)d->buf[d->cur] + (size_t)k * d->stride * d->elem;
    for (int64_t c0 = 0; c0 < n; c0 += (int64_t)chunk) {
      const int cnt = (int)std::min<int64_t>((int64_t)chunk, n - c0);
      HIP_OK(d, hipMemcpyAsync(d->stage, g + (size_t)k * n + c0, (size_t)cnt * 8,
                               hipMemcpyHostToDevice, d->stream));
      with_storage(d->p.storage, [&](auto tag) {
        using S = decltype(tag);
        set_plane_kernel<S><<<(cnt + 255) / 256, 256, 0, d->stream>>>(
            (S*)plane, d->flags, k, d->sigma, (int)c0, cnt, d->stage);
        return 0;
      });
      HIP_OK(d, hipGetLastError());
      HIP_OK(d, hipStreamSynchronize(d->stream));
    }
  }
  d->unstable = false;
  return LBM_OK;
}

LBM_API lbm_status lbm_get_state(lbm_domain d, double* g) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (!g) return fail(d, LBM_ERR_INVALID_ARG, "g is NULL");
  const int64_t n = d->geo.ncell;
  const size_t chunk = d->stage_cells * 4;
  for (int k = 0; k < kQ; ++k) {
    const char* plane = (const char*)d->buf[d->cur] + (size_t)k * d->stride * d->elem;
    for (int64_t c0 = 0; c0 < n; c0 += (int64_t)chunk) {
      const int cnt = (int)std::min<int64_t>((int64_t)chunk, n - c0);
      with_storage(d->p.storage, [&](auto tag) {
        using S = decltype(tag);
        get_plane_kernel<S><<<(cnt + 255) / 256, 256, 0, d->stream>>>(
            (const S*)plane, d->flags, k, d->sigma, (int)c0, cnt, d->stage);
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
  return enqueue_steps(d, n);
}

LBM_API lbm_status lbm_run_to_residual(lbm_domain d, double tol, int64_t max_steps,
                                       int64_t* steps_done, double* residual) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (max_steps < 0 || !(tol >= 0)) return fail(d, LBM_ERR_INVALID_ARG, "bad tol or max_steps");
  if (d->unstable) return fail(d, LBM_ERR_STATE, "state is unstable; re-initialise first");
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
          (const S*)d->buf[d->cur], d->flags, d->stride, d->sigma, (int)c0, cnt, d->stage);
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

LBM_API lbm_status lbm_mean_velocity(lbm_domain d, double U[3], double* max_speed,
                                     double* total_drho) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  double v[kRedVals];
  st = reduce_state(d, v);
  if (st != LBM_OK) return st;
  const double n = (double)d->geo.ncell;
  if (U) {
    U[0] = v[0] / n;
    U[1] = v[1] / n;
    U[2] = v[2] / n;
  }
  if (max_speed) *max_speed = v[5] > 0 ? NAN : std::sqrt(v[4]);
  if (total_drho) *total_drho = v[3];
  return LBM_OK;
}

// eq. (Darcy): K_D = mu U / |grad P| with mu = nu (rho0 = 1), |grad P| = dp/nx,
// dp = delta_rho / 3.
LBM_API lbm_status lbm_permeability(lbm_domain d, double* K_D, double* U_x) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (d->p.delta_rho == 0.0) return fail(d, LBM_ERR_STATE, "delta_rho is zero");
  double U[3];
  st = lbm_mean_velocity(d, U, nullptr, nullptr);
  if (st != LBM_OK) return st;
  const double dp = d->p.delta_rho / 3.0;
  if (K_D) *K_D = d->nu * U[0] * d->geo.nx / dp;
  if (U_x) *U_x = U[0];
  return LBM_OK;
}

LBM_API lbm_status lbm_drag(lbm_domain d, double F[3]) {
  lbm_status st = check_ready(d);
  if (st != LBM_OK) return st;
  if (!F) return fail(d, LBM_ERR_INVALID_ARG, "F is NULL");
  const StepParams sp = step_params(d);
  const bool cli = d->p.wall == LBM_WALL_CLI;
  with_storage(d->p.storage, [&](auto tag) {
    using S = decltype(tag);
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

LBM_API lbm_status lbm_set_delta_rho(lbm_domain d, double delta_rho) {
  if (!d) return LBM_ERR_INVALID_ARG;
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
