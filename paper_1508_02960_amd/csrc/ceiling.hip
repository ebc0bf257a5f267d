// Attainable-bandwidth probes (lbm_bandwidth_probe in include/lbm.h): plain
// streaming kernels of known byte counts that bound what the step kernel can
// reach on the GPU at hand, and that calibrate the HBM byte counters.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbm.h"

#define LBM_API extern "C" __attribute__((visibility("default")))

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

// Read and copy use the fastest instruction mix measured on MI355X (4 GiB,
// ms per pass): non-temporal loads, four 16-byte loads in flight per thread
// and 32768 workgroups.  Reads 6.4 -> 7.0 TB/s against ordinary loads; copies
// (non-temporal stores) 5.0 -> 5.5 TB/s.  The step kernel itself loses 29%
// with non-temporal loads (the lines its neighbouring pulls share are then
// dropped early), so these are ceilings for the memory system, not for its
// instruction mix.
constexpr int kBlocks = 32768, kThreads = 256, kUnroll = 4;

__global__ __launch_bounds__(kThreads) void read_kernel(const v4f* __restrict__ a, long long n4,
                                                        float* __restrict__ sink) {
  v4f s = {0.f, 0.f, 0.f, 0.f};
  for (long long i = blockIdx.x * (long long)(kThreads * kUnroll) + threadIdx.x; i < n4;
       i += (long long)gridDim.x * kThreads * kUnroll) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const long long j = i + (long long)u * kThreads;
      if (j < n4) s += __builtin_nontemporal_load(&a[j]);
    }
  }
  const float t = (s.x + s.y) + (s.z + s.w);
  if (t == -1.2345e-30f) sink[0] = t;  // keeps the loads; the data never sum to this
}

__global__ __launch_bounds__(kThreads) void write_kernel(v4f* __restrict__ b, long long n4) {
  const v4f v = {1.f, 2.f, 3.f, 4.f};
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n4;
       i += (long long)gridDim.x * kThreads)
    __builtin_nontemporal_store(v, &b[i]);
}

__global__ __launch_bounds__(kThreads) void copy_kernel(const v4f* __restrict__ a,
                                                        v4f* __restrict__ b, long long n4) {
  for (long long i = blockIdx.x * (long long)(kThreads * kUnroll) + threadIdx.x; i < n4;
       i += (long long)gridDim.x * kThreads * kUnroll) {
    v4f v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const long long j = i + (long long)u * kThreads;
      if (j < n4) v[u] = __builtin_nontemporal_load(&a[j]);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const long long j = i + (long long)u * kThreads;
      if (j < n4) __builtin_nontemporal_store(v[u], &b[j]);
    }
  }
}

// The step kernel's access pattern with nothing else: an all-fluid periodic
// cube of edge n in the step's layout for large FP32 states (16 x 4 tiles, n
// a multiple of 16; the 19 values of a tile stored as 19 runs of 64, one per
// direction); dst[k](x) = src[k](x - e_k), workgroups of 8 wavefronts over
// consecutive tiles of a z plane, non-temporal stores.
__constant__ int kEx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__constant__ int kEy[19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
__constant__ int kEz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};

__device__ __forceinline__ int xpart(int x) { return ((x >> 4) << 6) | (x & 15); }
__device__ __forceinline__ int ypart(int y, int ntx) { return (y >> 2) * (ntx << 6) + ((y & 3) << 4); }
__device__ __forceinline__ long long run_slot(int k, long long a) { return ((a >> 6) * 19 + k) * 64 + (a & 63); }

__global__ __launch_bounds__(512) void gather19_kernel(const float* __restrict__ src,
                                                       float* __restrict__ dst, int n) {
  const int ntx = n >> 4, nty = n >> 2, plane = n * n;
  const int tile = blockIdx.x * blockDim.y + threadIdx.y;
  if (tile >= ntx * nty) return;
  const int l = threadIdx.x;
  const int x = ((tile % ntx) << 4) + (l & 15), y = ((tile / ntx) << 2) + (l >> 4), z = blockIdx.z;
  // wrapped neighbour coordinates as address parts (index 0: -1, 1: 0, 2: +1)
  const int xs[3] = {xpart(x == 0 ? n - 1 : x - 1), xpart(x), xpart(x == n - 1 ? 0 : x + 1)};
  const int ys[3] = {ypart(y == 0 ? n - 1 : y - 1, ntx), ypart(y, ntx),
                     ypart(y == n - 1 ? 0 : y + 1, ntx)};
  const long long zs[3] = {(long long)(z == 0 ? n - 1 : z - 1) * plane, (long long)z * plane,
                           (long long)(z == n - 1 ? 0 : z + 1) * plane};
  const long long c = xs[1] + ys[1] + zs[1];
  float v[19];
#pragma unroll
  for (int k = 0; k < 19; ++k)
    v[k] = src[run_slot(k, xs[1 - kEx[k]] + ys[1 - kEy[k]] + zs[1 - kEz[k]])];
#pragma unroll
  for (int k = 0; k < 19; ++k) __builtin_nontemporal_store(v[k], &dst[run_slot(k, c)]);
}

}  // namespace

LBM_API lbm_status lbm_bandwidth_probe(int32_t kind, const void* src, void* dst, int64_t n,
                                       void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const bool a16 = ((uintptr_t)src & 15) == 0 && ((uintptr_t)dst & 15) == 0;
  switch (kind) {
    case LBM_PROBE_READ:
      if (!src || !dst || n <= 0 || n % 16 || !a16) return LBM_ERR_INVALID_ARG;
      read_kernel<<<kBlocks, kThreads, 0, s>>>((const v4f*)src, n / 16, (float*)dst);
      break;
    case LBM_PROBE_WRITE:
      if (!dst || n <= 0 || n % 16 || ((uintptr_t)dst & 15)) return LBM_ERR_INVALID_ARG;
      write_kernel<<<kBlocks, kThreads, 0, s>>>((v4f*)dst, n / 16);
      break;
    case LBM_PROBE_COPY:
      if (!src || !dst || n <= 0 || n % 16 || !a16) return LBM_ERR_INVALID_ARG;
      copy_kernel<<<kBlocks, kThreads, 0, s>>>((const v4f*)src, (v4f*)dst, n / 16);
      break;
    case LBM_PROBE_GATHER19: {
      if (!src || !dst || n < 16 || n % 16 || n > 1024 || !a16) return LBM_ERR_INVALID_ARG;
      const int e = (int)n, tiles = (e / 16) * (e / 4);
      gather19_kernel<<<dim3((tiles + 7) / 8, 1, e), dim3(64, 8), 0, s>>>(
          (const float*)src, (float*)dst, e);
      break;
    }
    default:
      return LBM_ERR_INVALID_ARG;
  }
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_ERR_DEVICE;
}
