// Kernels of the warm-start network: 3x3x3 convolutions with periodic
// (circular) padding as implicit GEMMs on BF16 MFMA (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation), plus the pooling, upsampling, activation, loss and
// optimiser kernels the network needs.  C ABI in include/lbm_nn.h.
//
// Tensors are channels-last: x[((n*D + z)*H + y)*W + x][c].  Convolution
// weights are w[co][tap][ci], tap = (dz+1)*9 + (dy+1)*3 + (dx+1).  BF16
// tensors are raw 16-bit patterns (uint16_t) on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>

#include "lbm_nn.h"

#define NN_API extern "C" __attribute__((visibility("default")))

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}
// round to nearest, ties to even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t b = __builtin_bit_cast(uint32_t, f);
  if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return (uint16_t)((b >> 16) | 0x40u);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

struct Shape {
  int n, d, h, w;
  long long m;  // n*d*h*w voxels
};

// voxel index -> (n, z, y, x)
__device__ __forceinline__ void unflatten(long long m, const Shape& s, int& n, int& z, int& y,
                                          int& x) {
  x = (int)(m % s.w);
  long long r = m / s.w;
  y = (int)(r % s.h);
  r /= s.h;
  z = (int)(r % s.d);
  n = (int)(r / s.d);
}

// voxel shifted by tap t with periodic wrap
__device__ __forceinline__ long long neighbour(int n, int z, int y, int x, int t, const Shape& s) {
  const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
  int zz = z + dz, yy = y + dy, xx = x + dx;
  zz = zz < 0 ? zz + s.d : (zz >= s.d ? zz - s.d : zz);
  yy = yy < 0 ? yy + s.h : (yy >= s.h ? yy - s.h : yy);
  xx = xx < 0 ? xx + s.w : (xx >= s.w ? xx - s.w : xx);
  return (((long long)n * s.d + zz) * s.h + yy) * s.w + xx;
}

// ---------------------------------------------------------------- forward
// y[m][co] = bias[co] + sum_{tap, ci} x[m + off(tap)][ci] * w[co][tap][ci]
// GEMM M = voxels, N = co, K = 27 ci (ci % 8 == 0).  Workgroup 256 threads
// = 4 wavefronts; tile 64 voxels x 64 output channels; K in chunks of 32.
// Wavefront wv computes voxel rows 16 wv .. 16 wv + 15 against the four
// 16-channel column blocks.  MFMA operands: lane l supplies row/column
// l % 16 and the 8 consecutive k of octet l / 16; the result holds rows
// 4 (l / 16) + i, column l % 16.
constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;

__global__ __launch_bounds__(256) void conv_fwd_kernel(const uint16_t* __restrict__ x,
                                                       const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias,
                                                       float* __restrict__ y, Shape s, int ci,
                                                       int co) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kBM][kBK + kPad];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN][kBK + kPad];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const long long m0 = (long long)blockIdx.x * kBM;
  const int n0 = blockIdx.y * kBN;
  const int K = 27 * ci;
  // this thread's load unit: row tid / 4, octet tid % 4
  const int lr = tid >> 2, lo = tid & 3;
  const long long lm = m0 + lr;
  int vn = 0, vz = 0, vy = 0, vx = 0;
  if (lm < s.m) unflatten(lm, s, vn, vz, vy, vx);
  const int wn = n0 + lr;

  f32x4 acc[4];
  for (int b = 0; b < 4; ++b) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < K; k0 += kBK) {
    const int k = k0 + lo * 8;
    uint4 av = make_uint4(0, 0, 0, 0), bv = make_uint4(0, 0, 0, 0);
    if (lm < s.m && k < K) {
      const int t = k / ci, c = k - t * ci;
      const long long nb = neighbour(vn, vz, vy, vx, t, s);
      av = *reinterpret_cast<const uint4*>(x + nb * ci + c);
    }
    if (wn < co && k < K) bv = *reinterpret_cast<const uint4*>(w + (long long)wn * K + k);
    *reinterpret_cast<uint4*>(&As[lr][lo * 8]) = av;
    *reinterpret_cast<uint4*>(&Bs[lr][lo * 8]) = bv;
    __syncthreads();
    const uint4 ar = *reinterpret_cast<const uint4*>(&As[wv * 16 + (lane & 15)][(lane >> 4) * 8]);
    const bf16x8 a = __builtin_bit_cast(bf16x8, ar);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (n0 + b * 16 < co) {
        const uint4 br = *reinterpret_cast<const uint4*>(&Bs[b * 16 + (lane & 15)][(lane >> 4) * 8]);
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, br),
                                                         acc[b], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int col = n0 + b * 16 + (lane & 15);
    if (col >= co) continue;
    const float bb = bias ? bias[col] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long long row = m0 + wv * 16 + (lane >> 4) * 4 + i;
      if (row < s.m) y[row * co + col] = acc[b][i] + bb;
    }
  }
}

// wt[ci][tap][co] = w[co][26 - tap][ci]: the backward-data convolution is the
// forward convolution of dy with these weights (mirrored taps, swapped roles).
__global__ void flip_weights_kernel(const uint16_t* __restrict__ w, uint16_t* __restrict__ wt,
                                    int ci, int co) {
  const long long n = 27LL * ci * co;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int o = (int)(i % co);
    const long long r = i / co;
    const int t = (int)(r % 27);
    const int c = (int)(r / 27);
    wt[i] = w[((long long)o * 27 + (26 - t)) * ci + c];
  }
}

// ------------------------------------------------------- backward weights
// dw[co][k] = sum_m dy[m][co] * x[m + off(tap(k))][ci(k)], split over voxel
// ranges: workgroup (tile of 64 co x 64 k, split s) writes its partial tile to
// part[s][co][k]; a second kernel folds the splits in order.  MFMA A operand =
// dy^T (co rows, m as the reduction), B operand = im2col(x) (m x k).
constexpr int kWM = 32;  // voxels per chunk

__global__ __launch_bounds__(256) void conv_bwdw_kernel(const uint16_t* __restrict__ x,
                                                        const uint16_t* __restrict__ dy,
                                                        float* __restrict__ part, Shape s, int ci,
                                                        int co, long long chunks_per_split) {
  __shared__ __attribute__((aligned(16))) uint16_t Ds[64][kWM + kPad];  // [co][m]
  __shared__ __attribute__((aligned(16))) uint16_t Xs[64][kWM + kPad];  // [k][m]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K = 27 * ci;
  const int c0 = blockIdx.x * 64;   // co tile
  const int kt0 = blockIdx.y * 64;  // k tile
  const int split = blockIdx.z;
  const long long mbeg = (long long)split * chunks_per_split * kWM;
  const long long mend = std::min<long long>(s.m, mbeg + chunks_per_split * kWM);
  f32x4 acc[4];
  for (int b = 0; b < 4; ++b) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
  // load units: dy tile 32 m x 64 co = 256 octets (m = tid / 8, co octet tid % 8)
  //             x tile  32 m x 64 k  = 256 octets (m = tid / 8, k octet tid % 8)
  const int um = tid >> 3, uo = tid & 7;
  for (long long mc = mbeg; mc < mend; mc += kWM) {
    const long long m = mc + um;
    uint4 dv = make_uint4(0, 0, 0, 0), xv = make_uint4(0, 0, 0, 0);
    if (m < mend) {
      const int cc = c0 + uo * 8;
      if (cc < co) dv = *reinterpret_cast<const uint4*>(dy + m * co + cc);
      const int k = kt0 + uo * 8;
      if (k < K) {
        int vn, vz, vy, vx;
        unflatten(m, s, vn, vz, vy, vx);
        const int t = k / ci, c = k - t * ci;
        xv = *reinterpret_cast<const uint4*>(x + neighbour(vn, vz, vy, vx, t, s) * ci + c);
      }
    }
    // transpose into LDS: element e of the octet goes to row (octet*8 + e), column um
    const uint16_t* dp = reinterpret_cast<const uint16_t*>(&dv);
    const uint16_t* xp = reinterpret_cast<const uint16_t*>(&xv);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      Ds[uo * 8 + e][um] = dp[e];
      Xs[uo * 8 + e][um] = xp[e];
    }
    __syncthreads();
    if (c0 + wv * 16 < co) {
      const uint4 ar = *reinterpret_cast<const uint4*>(&Ds[wv * 16 + (lane & 15)][(lane >> 4) * 8]);
      const bf16x8 a = __builtin_bit_cast(bf16x8, ar);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint4 br = *reinterpret_cast<const uint4*>(&Xs[b * 16 + (lane & 15)][(lane >> 4) * 8]);
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, br),
                                                         acc[b], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  float* out = part + (long long)split * co * K;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int k = kt0 + b * 16 + (lane & 15);
    if (k >= K) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = c0 + wv * 16 + (lane >> 4) * 4 + i;
      if (o < co) out[(long long)o * K + k] = acc[b][i];
    }
  }
}

__global__ void fold_splits_kernel(const float* __restrict__ part, float* __restrict__ dw,
                                   long long n, int splits) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    float a = 0.f;
    for (int s = 0; s < splits; ++s) a += part[(long long)s * n + i];
    dw[i] = a;
  }
}

// db[c] = sum_m dy[m][c] (fixed order per channel, block per channel)
__global__ __launch_bounds__(256) void bias_grad_kernel(const float* __restrict__ dy,
                                                        float* __restrict__ db, long long m,
                                                        int c) {
  __shared__ float sh[256];
  const int ch = blockIdx.x;
  float a = 0.f;
  for (long long i = threadIdx.x; i < m; i += 256) a += dy[i * c + ch];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[ch] = sh[0];
}

// --------------------------------------------------------------- elementwise

__global__ void relu_fwd_kernel(const float* __restrict__ z, uint16_t* __restrict__ a,
                                long long n, int relu) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    a[i] = f2bf(relu ? fmaxf(z[i], 0.f) : z[i]);
}

// dz = da where the stored activation is positive
__global__ void relu_bwd_kernel(const float* __restrict__ da, const uint16_t* __restrict__ a,
                                float* __restrict__ dz, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dz[i] = bf2f(a[i]) > 0.f ? da[i] : 0.f;
}

__global__ void cast_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y,
                                 long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = f2bf(x[i]);
}

// 2x2x2 average pooling (fine shape s, coarse = halves), bf16 in/out
__global__ void pool_fwd_kernel(const uint16_t* __restrict__ x, uint16_t* __restrict__ y, Shape s,
                                int c) {
  const Shape q{s.n, s.d / 2, s.h / 2, s.w / 2, s.m / 8};
  const long long n = q.m * c;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c);
    int vn, vz, vy, vx;
    unflatten(i / c, q, vn, vz, vy, vx);
    float a = 0.f;
    for (int o = 0; o < 8; ++o) {
      const long long f = (((long long)vn * s.d + 2 * vz + (o >> 2)) * s.h + 2 * vy + ((o >> 1) & 1)) *
                              s.w + 2 * vx + (o & 1);
      a += bf2f(x[f * c + ch]);
    }
    y[i] = f2bf(0.125f * a);
  }
}

// gradient of the average pooling: each fine voxel gets 1/8 of its parent
__global__ void pool_bwd_kernel(const float* __restrict__ dy, float* __restrict__ dx, Shape s,
                                int c) {
  const Shape q{s.n, s.d / 2, s.h / 2, s.w / 2, s.m / 8};
  const long long n = s.m * c;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c);
    int vn, vz, vy, vx;
    unflatten(i / c, s, vn, vz, vy, vx);
    const long long p = (((long long)vn * q.d + vz / 2) * q.h + vy / 2) * q.w + vx / 2;
    dx[i] = 0.125f * dy[p * c + ch];
  }
}

// nearest-neighbour upsampling x2 (coarse shape q -> fine), bf16 in/out
__global__ void up_fwd_kernel(const uint16_t* __restrict__ x, uint16_t* __restrict__ y, Shape q,
                              int c) {
  const Shape s{q.n, q.d * 2, q.h * 2, q.w * 2, q.m * 8};
  const long long n = s.m * c;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c);
    int vn, vz, vy, vx;
    unflatten(i / c, s, vn, vz, vy, vx);
    const long long p = (((long long)vn * q.d + vz / 2) * q.h + vy / 2) * q.w + vx / 2;
    y[i] = x[p * c + ch];
  }
}

// gradient of the upsampling: sum over the 8 fine children
__global__ void up_bwd_kernel(const float* __restrict__ dy, float* __restrict__ dx, Shape q,
                              int c) {
  const Shape s{q.n, q.d * 2, q.h * 2, q.w * 2, q.m * 8};
  const long long n = q.m * c;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c);
    int vn, vz, vy, vx;
    unflatten(i / c, q, vn, vz, vy, vx);
    float a = 0.f;
    for (int o = 0; o < 8; ++o) {
      const long long f = (((long long)vn * s.d + 2 * vz + (o >> 2)) * s.h + 2 * vy + ((o >> 1) & 1)) *
                              s.w + 2 * vx + (o & 1);
      a += dy[f * c + ch];
    }
    dx[i] = a;
  }
}

// y = [a | b] along channels (bf16)
__global__ void concat_kernel(const uint16_t* __restrict__ a, const uint16_t* __restrict__ b,
                              uint16_t* __restrict__ y, long long m, int ca, int cb) {
  const int c = ca + cb;
  const long long n = m * c;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long v = i / c;
    const int ch = (int)(i % c);
    y[i] = ch < ca ? a[v * ca + ch] : b[v * cb + ch - ca];
  }
}

// da, db = split of dy along channels (fp32); either output may be null
__global__ void split_kernel(const float* __restrict__ dy, float* __restrict__ da,
                             float* __restrict__ db, long long m, int ca, int cb) {
  const int c = ca + cb;
  const long long n = m * c;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long v = i / c;
    const int ch = (int)(i % c);
    if (ch < ca) {
      if (da) da[v * ca + ch] = dy[i];
    } else if (db) {
      db[v * cb + ch - ca] = dy[i];
    }
  }
}

__global__ void add_kernel(float* __restrict__ y, const float* __restrict__ x, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] += x[i];
}

// Masked mean-squared error over the first `used` of c channels at voxels
// with weight[m] > 0: loss partials per block (fixed tree), gradient
// 2 (pred - target) weight / norm.
__global__ __launch_bounds__(256) void mse_kernel(const float* __restrict__ pred,
                                                  const float* __restrict__ target,
                                                  const float* __restrict__ weight,
                                                  float* __restrict__ grad,
                                                  double* __restrict__ partial, long long m, int c,
                                                  int used, double inv_norm) {
  __shared__ double sh[256];
  double a = 0.0;
  const long long n = m * c;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long v = i / c;
    const int ch = (int)(i % c);
    float g = 0.f;
    if (ch < used && weight[v] > 0.f) {
      const float d = pred[i] - target[v * used + ch];
      a += (double)d * d * weight[v];
      g = (float)(2.0 * d * weight[v] * inv_norm);
    }
    grad[i] = g;
  }
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] * inv_norm;
}

// Adam update of FP32 master weights, refreshing the BF16 copy.
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m1, float* __restrict__ m2,
                            uint16_t* __restrict__ wb, long long n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float wi = w[i] - lr * (a * c1) / (sqrtf(b * c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = f2bf(wi);
  }
}

int grid_for(long long n) { return (int)std::min<long long>((n + 255) / 256, 8192); }

lbm_status check_launch() {
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_ERR_DEVICE;
}

Shape shape_of(int n, int d, int h, int w) {
  return Shape{n, d, h, w, (long long)n * d * h * w};
}

bool bad_shape(int n, int d, int h, int w) { return n < 1 || d < 1 || h < 1 || w < 1; }

}  // namespace

// ------------------------------------------------------------------ C ABI

NN_API lbm_status nn_conv3d_forward(const void* x, const void* w, const float* bias, float* y,
                                    int n, int d, int h, int wd, int ci, int co, void* stream) {
  if (!x || !w || !y || bad_shape(n, d, h, wd) || ci < 8 || ci % 8 || co < 1)
    return LBM_ERR_INVALID_ARG;
  const Shape s = shape_of(n, d, h, wd);
  dim3 grid((unsigned)((s.m + kBM - 1) / kBM), (unsigned)((co + kBN - 1) / kBN));
  conv_fwd_kernel<<<grid, 256, 0, (hipStream_t)stream>>>((const uint16_t*)x, (const uint16_t*)w,
                                                         bias, y, s, ci, co);
  return check_launch();
}

NN_API lbm_status nn_conv3d_flip_weights(const void* w, void* wt, int ci, int co, void* stream) {
  if (!w || !wt || ci < 1 || co < 1) return LBM_ERR_INVALID_ARG;
  flip_weights_kernel<<<grid_for(27LL * ci * co), 256, 0, (hipStream_t)stream>>>(
      (const uint16_t*)w, (uint16_t*)wt, ci, co);
  return check_launch();
}

NN_API lbm_status nn_conv3d_backward_data(const void* dy, const void* wt, float* dx, int n, int d,
                                          int h, int wd, int ci, int co, void* stream) {
  // forward convolution of dy (co channels) with the flipped weights (ci outputs)
  return nn_conv3d_forward(dy, wt, nullptr, dx, n, d, h, wd, co, ci, stream);
}

NN_API lbm_status nn_conv3d_backward_weight_workspace(int n, int d, int h, int wd, int ci, int co,
                                                      size_t* bytes, int* splits) {
  if (!bytes || bad_shape(n, d, h, wd) || ci < 8 || ci % 8 || co < 8 || co % 8)
    return LBM_ERR_INVALID_ARG;
  const long long m = (long long)n * d * h * wd;
  const long long tiles = (long long)((co + 63) / 64) * ((27 * ci + 63) / 64);
  const long long chunks = (m + kWM - 1) / kWM;
  long long sp = std::max<long long>(1, std::min<long long>(chunks, 2048 / std::max<long long>(tiles, 1)));
  sp = std::min<long long>(sp, 256);
  *bytes = (size_t)sp * co * 27 * ci * sizeof(float);
  if (splits) *splits = (int)sp;
  return LBM_OK;
}

NN_API lbm_status nn_conv3d_backward_weight(const void* x, const void* dy, float* dw, void* ws,
                                            size_t ws_bytes, int n, int d, int h, int wd, int ci,
                                            int co, void* stream) {
  size_t need = 0;
  int sp = 0;
  lbm_status st = nn_conv3d_backward_weight_workspace(n, d, h, wd, ci, co, &need, &sp);
  if (st != LBM_OK) return st;
  if (!x || !dy || !dw || !ws || ws_bytes < need) return LBM_ERR_WORKSPACE;
  const Shape s = shape_of(n, d, h, wd);
  const long long chunks = (s.m + kWM - 1) / kWM;
  const long long per = (chunks + sp - 1) / sp;
  dim3 grid((unsigned)((co + 63) / 64), (unsigned)((27 * ci + 63) / 64), (unsigned)sp);
  conv_bwdw_kernel<<<grid, 256, 0, (hipStream_t)stream>>>((const uint16_t*)x, (const uint16_t*)dy,
                                                          (float*)ws, s, ci, co, per);
  const long long nw = (long long)co * 27 * ci;
  fold_splits_kernel<<<grid_for(nw), 256, 0, (hipStream_t)stream>>>((const float*)ws, dw, nw, sp);
  return check_launch();
}

NN_API lbm_status nn_bias_grad(const float* dy, float* db, long long m, int c, void* stream) {
  if (!dy || !db || m < 1 || c < 1) return LBM_ERR_INVALID_ARG;
  bias_grad_kernel<<<c, 256, 0, (hipStream_t)stream>>>(dy, db, m, c);
  return check_launch();
}

NN_API lbm_status nn_activation_forward(const float* z, void* a, long long n, int relu,
                                        void* stream) {
  if (!z || !a || n < 0) return LBM_ERR_INVALID_ARG;
  relu_fwd_kernel<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(z, (uint16_t*)a, n, relu);
  return check_launch();
}

NN_API lbm_status nn_relu_backward(const float* da, const void* a, float* dz, long long n,
                                   void* stream) {
  if (!da || !a || !dz || n < 0) return LBM_ERR_INVALID_ARG;
  relu_bwd_kernel<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(da, (const uint16_t*)a, dz, n);
  return check_launch();
}

NN_API lbm_status nn_cast_bf16(const float* x, void* y, long long n, void* stream) {
  if (!x || !y || n < 0) return LBM_ERR_INVALID_ARG;
  cast_bf16_kernel<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(x, (uint16_t*)y, n);
  return check_launch();
}

NN_API lbm_status nn_pool2_forward(const void* x, void* y, int n, int d, int h, int w, int c,
                                   void* stream) {
  if (!x || !y || bad_shape(n, d, h, w) || d % 2 || h % 2 || w % 2 || c < 1)
    return LBM_ERR_INVALID_ARG;
  const Shape s = shape_of(n, d, h, w);
  pool_fwd_kernel<<<grid_for(s.m / 8 * c), 256, 0, (hipStream_t)stream>>>(
      (const uint16_t*)x, (uint16_t*)y, s, c);
  return check_launch();
}

NN_API lbm_status nn_pool2_backward(const float* dy, float* dx, int n, int d, int h, int w, int c,
                                    void* stream) {
  if (!dy || !dx || bad_shape(n, d, h, w) || d % 2 || h % 2 || w % 2 || c < 1)
    return LBM_ERR_INVALID_ARG;
  const Shape s = shape_of(n, d, h, w);
  pool_bwd_kernel<<<grid_for(s.m * c), 256, 0, (hipStream_t)stream>>>(dy, dx, s, c);
  return check_launch();
}

NN_API lbm_status nn_upsample2_forward(const void* x, void* y, int n, int d, int h, int w, int c,
                                       void* stream) {
  if (!x || !y || bad_shape(n, d, h, w) || c < 1) return LBM_ERR_INVALID_ARG;
  const Shape q = shape_of(n, d, h, w);
  up_fwd_kernel<<<grid_for(q.m * 8 * c), 256, 0, (hipStream_t)stream>>>(
      (const uint16_t*)x, (uint16_t*)y, q, c);
  return check_launch();
}

NN_API lbm_status nn_upsample2_backward(const float* dy, float* dx, int n, int d, int h, int w,
                                        int c, void* stream) {
  if (!dy || !dx || bad_shape(n, d, h, w) || c < 1) return LBM_ERR_INVALID_ARG;
  const Shape q = shape_of(n, d, h, w);
  up_bwd_kernel<<<grid_for(q.m * c), 256, 0, (hipStream_t)stream>>>(dy, dx, q, c);
  return check_launch();
}

NN_API lbm_status nn_concat_channels(const void* a, const void* b, void* y, long long m, int ca,
                                     int cb, void* stream) {
  if (!a || !b || !y || m < 1 || ca < 1 || cb < 1) return LBM_ERR_INVALID_ARG;
  concat_kernel<<<grid_for(m * (ca + cb)), 256, 0, (hipStream_t)stream>>>(
      (const uint16_t*)a, (const uint16_t*)b, (uint16_t*)y, m, ca, cb);
  return check_launch();
}

NN_API lbm_status nn_split_channels(const float* dy, float* da, float* db, long long m, int ca,
                                    int cb, void* stream) {
  if (!dy || m < 1 || ca < 1 || cb < 1) return LBM_ERR_INVALID_ARG;
  split_kernel<<<grid_for(m * (ca + cb)), 256, 0, (hipStream_t)stream>>>(dy, da, db, m, ca, cb);
  return check_launch();
}

NN_API lbm_status nn_add(float* y, const float* x, long long n, void* stream) {
  if (!y || !x || n < 0) return LBM_ERR_INVALID_ARG;
  add_kernel<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(y, x, n);
  return check_launch();
}

NN_API lbm_status nn_masked_mse(const float* pred, const float* target, const float* weight,
                                float* grad, double* partial, int n_partial, long long m, int c,
                                int used, double norm, void* stream) {
  if (!pred || !target || !weight || !grad || !partial || n_partial < 1 || m < 1 || used > c ||
      !(norm > 0))
    return LBM_ERR_INVALID_ARG;
  mse_kernel<<<n_partial, 256, 0, (hipStream_t)stream>>>(pred, target, weight, grad, partial, m, c,
                                                         used, 1.0 / norm);
  return check_launch();
}

NN_API lbm_status nn_adam(float* w, const float* g, float* m1, float* m2, void* w_bf16, long long n,
                          float lr, float b1, float b2, float eps, int step, void* stream) {
  if (!w || !g || !m1 || !m2 || n < 0 || step < 1) return LBM_ERR_INVALID_ARG;
  const float c1 = 1.f / (1.f - powf(b1, (float)step)), c2 = 1.f / (1.f - powf(b2, (float)step));
  adam_kernel<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(w, g, m1, m2, (uint16_t*)w_bf16, n, lr,
                                                            b1, b2, eps, c1, c2);
  return check_launch();
}
