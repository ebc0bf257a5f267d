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

// Output of a forward convolution: the FP32 pre-activation y, or (ACT) the
// BF16 activation a = bf16(relu ? max(y, 0) : y) that the next layer reads,
// without the FP32 round trip through memory.
template <bool ACT>
__device__ __forceinline__ void store_out(void* out, long long i, float v, int relu) {
  if constexpr (ACT)
    static_cast<uint16_t*>(out)[i] = f2bf(relu ? fmaxf(v, 0.f) : v);
  else
    static_cast<float*>(out)[i] = v;
}

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
// y[m][co] = bias[co] + sum_{tap, ci} x[m + off(tap)][ci] * w[co][tap][ci]:
// an implicit GEMM with M = voxels, N = co and K = 27 ci (ci % 8 == 0).  MFMA
// operands (v_mfma_f32_16x16x32_bf16): lane l supplies row/column l % 16 and
// the 8 consecutive k of octet l / 16; the result holds rows 4 (l / 16) + i,
// column l % 16.
constexpr int kPad = 8;

// Tiled forward convolution: block tile 128 voxels x BN output channels
// (BN = 16, 32 or 64), K = 27 ci staged 64 at a time through LDS.  Each of
// the 4 wavefronts owns 32 voxel rows (two 16-row MFMA tiles) against all
// BN/16 column tiles.  The 27 neighbour voxels of the block's 128 rows are
// tabulated in LDS once, so the gather of a K stage is a table lookup plus
// the tap/channel position of the thread's 8-element granule, advanced
// incrementally.  The next stage's global loads are issued into registers
// before the current stage's MFMAs (one stage of prefetch).
template <int BN, bool ACT>
__global__ __launch_bounds__(256) void conv_fwd_tiled_kernel(const uint16_t* __restrict__ x,
                                                             const uint16_t* __restrict__ w,
                                                             const float* __restrict__ bias,
                                                             void* __restrict__ y, Shape s,
                                                             int ci, int co, int relu) {
  constexpr int BM = 128, BK = 64, LD = BK + 8;
  constexpr int NBG = BN * BK / 8;          // B granules per stage
  constexpr int NB = (NBG + 255) / 256;     // B granules per thread (at most)
  constexpr int NT = BN / 16;               // column tiles
  __shared__ __attribute__((aligned(16))) uint16_t As[BM * LD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LD];
  __shared__ int nbr[27 * BM];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const long long m0 = (long long)blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  const int K = 27 * ci;
  for (int i = tid; i < 27 * BM; i += 256) {
    const int t = i / BM, r = i - t * BM;
    const long long m = m0 + r;
    int v = -1;
    if (m < s.m) {
      int vn, vz, vy, vx;
      unflatten(m, s, vn, vz, vy, vx);
      v = (int)neighbour(vn, vz, vy, vx, t, s);
    }
    nbr[i] = v;
  }
  // this thread's granules: rows (tid >> 3) + 32 i of A, B rows from g = tid + 256 i,
  // all at K offset koff = 8 (tid & 7) within the stage
  const int koff = 8 * (tid & 7);
  int ta = 0, ca = koff;
  while (ca >= ci) {
    ca -= ci;
    ++ta;
  }
  __syncthreads();

  uint4 ra[4], rb[NB];
  auto gload = [&](int k0) {
    const bool kin = k0 + koff < K;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ra[i] = make_uint4(0, 0, 0, 0);
      if (kin) {
        const int v = nbr[ta * BM + (tid >> 3) + 32 * i];
        if (v >= 0) ra[i] = *reinterpret_cast<const uint4*>(x + (long long)v * ci + ca);
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int g = tid + 256 * i;
      const int col = n0 + (g >> 3);
      rb[i] = make_uint4(0, 0, 0, 0);
      if (g < NBG && kin && col < co)
        rb[i] = *reinterpret_cast<const uint4*>(w + (long long)col * K + k0 + koff);
    }
  };
  f32x4 acc[2][NT];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[r][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  gload(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      *reinterpret_cast<uint4*>(&As[((tid >> 3) + 32 * i) * LD + koff]) = ra[i];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int g = tid + 256 * i;
      if (g < NBG) *reinterpret_cast<uint4*>(&Bs[(g >> 3) * LD + koff]) = rb[i];
    }
    __syncthreads();
    if (k0 + BK < K) {
      ca += BK;
      while (ca >= ci) {
        ca -= ci;
        ++ta;
      }
      gload(k0 + BK);
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 32) {
      const int kk = ks + 8 * (lane >> 4);
      const bf16x8 a0 = __builtin_bit_cast(
          bf16x8, *reinterpret_cast<const uint4*>(&As[(wv * 32 + (lane & 15)) * LD + kk]));
      const bf16x8 a1 = __builtin_bit_cast(
          bf16x8, *reinterpret_cast<const uint4*>(&As[(wv * 32 + 16 + (lane & 15)) * LD + kk]));
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const bf16x8 bf = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const uint4*>(&Bs[(b * 16 + (lane & 15)) * LD + kk]));
        acc[0][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bf, acc[0][b], 0, 0, 0);
        acc[1][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bf, acc[1][b], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    const int col = n0 + b * 16 + (lane & 15);
    if (col >= co) continue;
    const float bb = bias ? bias[col] : 0.f;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long row = m0 + wv * 32 + r * 16 + (lane >> 4) * 4 + i;
        if (row < s.m) store_out<ACT>(y, row * co + col, acc[r][b][i] + bb, relu);
      }
  }
}

// Spatially tiled forward convolution for ci % 32 == 0 and box edges that
// are multiples of the tile: each block computes a 4 x 8 x 8 voxel tile
// (z, y, x; 256 rows of the implicit GEMM) against BN output channels.  The
// input is taken 32 channels at a time: the 6 x 10 x 10 halo of the tile
// (periodic wrap) is staged in LDS once per chunk, so each input voxel is
// fetched about 2.3 times instead of once per tap, and the 27 taps read
// their A operands from LDS at shifted halo positions.  Wavefront wv owns
// the z layer wv of the tile (64 rows = 4 MFMA row tiles); B operands (the
// weights of one tap and 32 channels) come from global memory (L1/L2
// resident), one tap ahead.
constexpr int kTZ = 4, kTY = 8, kTX = 8;
constexpr int kHZ = kTZ + 2, kHY = kTY + 2, kHX = kTX + 2;
constexpr int kHalo = kHZ * kHY * kHX;  // 600 voxels
constexpr int kCC = 32;                 // channels per chunk
constexpr int kHLD = kCC + 8;           // LDS row stride (halfs) of a halo voxel

template <int BN, bool ACT>
__global__ __launch_bounds__(256) void conv_fwd_spatial_kernel(const uint16_t* __restrict__ x,
                                                               const uint16_t* __restrict__ w,
                                                               const float* __restrict__ bias,
                                                               void* __restrict__ y, Shape s,
                                                               int ci, int co, int relu) {
  constexpr int NT = BN / 16;
  __shared__ __attribute__((aligned(16))) uint16_t Hs[kHalo * kHLD];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // tile position
  const int tx_n = s.w / kTX, ty_n = s.h / kTY, tz_n = s.d / kTZ;
  long long t = blockIdx.x;
  const int bx = (int)(t % tx_n);
  t /= tx_n;
  const int by = (int)(t % ty_n);
  t /= ty_n;
  const int bz = (int)(t % tz_n);
  const int bn_ = (int)(t / tz_n);
  const int x0 = bx * kTX, y0 = by * kTY, z0 = bz * kTZ;
  const int n0 = blockIdx.y * BN;
  const int K = 27 * ci;
  // the lane's rows: row tile rt holds tile rows 16 rt + (lane & 15), i.e.
  // (tz, ty, tx) = (wv, 2 rt + (lane & 15) / 8, lane & 7)
  const int lx = lane & 7, ly = (lane & 15) >> 3, oct = lane >> 4;

  f32x4 acc[4][NT];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[r][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int c0 = 0; c0 < ci; c0 += kCC) {
    __syncthreads();  // the previous chunk's reads are done
    for (int g = tid; g < kHalo * (kCC / 8); g += 256) {
      const int hv = g >> 2, part = g & 3;
      const int hz = hv / (kHY * kHX), hy = (hv / kHX) % kHY, hx = hv % kHX;
      int zz = z0 + hz - 1, yy = y0 + hy - 1, xx = x0 + hx - 1;
      zz = zz < 0 ? zz + s.d : (zz >= s.d ? zz - s.d : zz);
      yy = yy < 0 ? yy + s.h : (yy >= s.h ? yy - s.h : yy);
      xx = xx < 0 ? xx + s.w : (xx >= s.w ? xx - s.w : xx);
      const long long v = (((long long)bn_ * s.d + zz) * s.h + yy) * s.w + xx;
      *reinterpret_cast<uint4*>(&Hs[hv * kHLD + 8 * part]) =
          *reinterpret_cast<const uint4*>(x + v * ci + c0 + 8 * part);
    }
    __syncthreads();
    // B fragments of tap 0, then one tap ahead
    uint4 bq[NT];
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      const int col = n0 + b * 16 + (lane & 15);
      bq[b] = col < co ? *reinterpret_cast<const uint4*>(w + (long long)col * K + c0 + 8 * oct)
                       : make_uint4(0, 0, 0, 0);
    }
    for (int tap = 0; tap < 27; ++tap) {
      bf16x8 bf[NT];
#pragma unroll
      for (int b = 0; b < NT; ++b) bf[b] = __builtin_bit_cast(bf16x8, bq[b]);
      if (tap + 1 < 27) {
#pragma unroll
        for (int b = 0; b < NT; ++b) {
          const int col = n0 + b * 16 + (lane & 15);
          bq[b] = col < co ? *reinterpret_cast<const uint4*>(
                                 w + (long long)col * K + (long long)(tap + 1) * ci + c0 + 8 * oct)
                           : make_uint4(0, 0, 0, 0);
        }
      }
      const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;  // halo offsets 0..2
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        const int hv = ((wv + dz) * kHY + (2 * rt + ly + dy)) * kHX + (lx + dx);
        const bf16x8 a = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const uint4*>(&Hs[hv * kHLD + 8 * oct]));
#pragma unroll
        for (int b = 0; b < NT; ++b)
          acc[rt][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bf[b], acc[rt][b], 0, 0, 0);
      }
    }
  }
  // result rows 4 (lane / 16) + i of row tile rt, column lane & 15
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    const int col = n0 + b * 16 + (lane & 15);
    if (col >= co) continue;
    const float bb = bias ? bias[col] : 0.f;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * rt + 4 * oct + i;  // row within the wavefront's z layer
        const int tyy = r >> 3, txx = r & 7;
        const long long v =
            (((long long)bn_ * s.d + z0 + wv) * s.h + y0 + tyy) * s.w + x0 + txx;
        store_out<ACT>(y, v * co + col, acc[rt][b][i] + bb, relu);
      }
  }
}

// Spatially tiled weight gradient for boxes that are multiples of the
// 4 x 8 x 8 tile: dw[co][tap][ci] = sum over the voxels v of dy[v][co]
// x[v + off(tap)][ci], an MFMA GEMM whose K runs over the 256 voxels of a
// tile.  Block (g, chunk, co tile) adds up the tiles g, g + G, g + 2G, ...
// (a fixed order) for 16 CT input and 16 RT output channels (channels past
// ci or co are zero) and writes its sum to part[g]; fold_splits_kernel adds
// the G partials in order, so the result is deterministic.  Per tile, LDS
// holds dy transposed (Ds[co][voxel]) and three copies of the 6 x 10 x 10
// input halo shifted by dx = 0, 1, 2, channel-major (Xs[dx][c][hz][hy][tx]),
// so that both MFMA operands are 8 consecutive voxels (one x row of the
// tile) read as one aligned 16-byte word.  Wavefront wv owns the taps wv,
// wv + 4, ...
constexpr int kXR = kHZ * kHY * kTX;       // halo positions of one shifted copy of a channel
constexpr int kDLD = kTZ * kTY * kTX + 8;  // Ds row stride (halfs)

__device__ __forceinline__ void unpack8(uint4 u, uint16_t (&h)[8]) {
  h[0] = (uint16_t)u.x;
  h[1] = (uint16_t)(u.x >> 16);
  h[2] = (uint16_t)u.y;
  h[3] = (uint16_t)(u.y >> 16);
  h[4] = (uint16_t)u.z;
  h[5] = (uint16_t)(u.z >> 16);
  h[6] = (uint16_t)u.w;
  h[7] = (uint16_t)(u.w >> 16);
}

template <int RT, int CT>
__global__ __launch_bounds__(256) void conv_bwdw_spatial_kernel(const uint16_t* __restrict__ x,
                                                                const uint16_t* __restrict__ dy,
                                                                float* __restrict__ part, Shape s,
                                                                int ci, int co, int tiles) {
  constexpr int CC = 16 * CT, OC = 16 * RT;  // input / output channels of the block
  __shared__ __attribute__((aligned(16))) uint16_t Xs[3 * CC * kXR];
  __shared__ __attribute__((aligned(16))) uint16_t Ds[OC * kDLD];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, oct = lane >> 4;
  const int G = gridDim.x, c0 = blockIdx.y * CC, o0 = blockIdx.z * OC;
  const int tx_n = s.w / kTX, ty_n = s.h / kTY, tz_n = s.d / kTZ;
  f32x4 acc[7][RT][CT];
#pragma unroll
  for (int j = 0; j < 7; ++j)
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[j][r][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int t = blockIdx.x; t < tiles; t += G) {
    int q = t;
    const int bx = q % tx_n;
    q /= tx_n;
    const int by = q % ty_n;
    q /= ty_n;
    const int bz = q % tz_n;
    const int bn_ = q / tz_n;
    const int x0 = bx * kTX, y0 = by * kTY, z0 = bz * kTZ;
    __syncthreads();  // the previous tile's reads are done
    for (int g = tid; g < kHalo * (CC / 8); g += 256) {
      const int hv = g / (CC / 8), p8 = 8 * (g % (CC / 8));
      const int hz = hv / (kHY * kHX), hy = (hv / kHX) % kHY, hx = hv % kHX;
      int zz = z0 + hz - 1, yy = y0 + hy - 1, xx = x0 + hx - 1;
      zz = zz < 0 ? zz + s.d : (zz >= s.d ? zz - s.d : zz);
      yy = yy < 0 ? yy + s.h : (yy >= s.h ? yy - s.h : yy);
      xx = xx < 0 ? xx + s.w : (xx >= s.w ? xx - s.w : xx);
      const long long v = (((long long)bn_ * s.d + zz) * s.h + yy) * s.w + xx;
      uint16_t h[8];
      unpack8(c0 + p8 < ci ? *reinterpret_cast<const uint4*>(x + v * ci + c0 + p8)
                           : make_uint4(0, 0, 0, 0),
              h);
      const int pos = (hz * kHY + hy) * kTX;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int tx = hx - dx;
        if (tx < 0 || tx >= kTX) continue;
#pragma unroll
        for (int i = 0; i < 8; ++i) Xs[(dx * CC + p8 + i) * kXR + pos + tx] = h[i];
      }
    }
    for (int g = tid; g < kTZ * kTY * kTX * (OC / 8); g += 256) {
      const int r = g / (OC / 8), p8 = 8 * (g % (OC / 8));
      const int tz = r >> 6, ty = (r >> 3) & 7, tx = r & 7;
      const long long v = (((long long)bn_ * s.d + z0 + tz) * s.h + y0 + ty) * s.w + x0 + tx;
      uint16_t h[8];
      unpack8(o0 + p8 < co ? *reinterpret_cast<const uint4*>(dy + v * co + o0 + p8)
                           : make_uint4(0, 0, 0, 0),
              h);
#pragma unroll
      for (int i = 0; i < 8; ++i) Ds[(p8 + i) * kDLD + r] = h[i];
    }
    __syncthreads();
#pragma unroll 2
    for (int ks = 0; ks < 8; ++ks) {
      const int vr = 4 * ks + oct;  // x row (tz, ty) of this lane's 8 voxels
      const int tz = vr >> 3, ty = vr & 7;
      bf16x8 a[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        a[rt] = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const uint4*>(&Ds[(16 * rt + (lane & 15)) * kDLD + 8 * vr]));
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        const int tap = wv + 4 * j;
        if (tap >= 27) continue;
        const int dz = tap / 9, dyy = (tap / 3) % 3, dx = tap % 3;
        const int pos = ((tz + dz) * kHY + ty + dyy) * kTX;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const bf16x8 b = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const uint4*>(
                          &Xs[(dx * CC + 16 * ct + (lane & 15)) * kXR + pos]));
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
            acc[j][rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt], b, acc[j][rt][ct], 0, 0, 0);
        }
      }
    }
  }
  // result rows (co) 4 (lane / 16) + i of row tile rt, column (ci) lane & 15
  const long long base = (long long)blockIdx.x * co * 27 * ci;
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const int tap = wv + 4 * j;
    if (tap >= 27) continue;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int o = o0 + 16 * rt + 4 * oct + i, c = c0 + 16 * ct + (lane & 15);
          if (o < co && c < ci) part[base + ((long long)o * 27 + tap) * ci + c] = acc[j][rt][ct][i];
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
constexpr int kWM = 64;  // voxels per stage

// Voxel coordinates advanced by `step` voxels (row-major n, z, y, x).
__device__ __forceinline__ void advance_voxel(int& n, int& z, int& y, int& x, int step,
                                              const Shape& s) {
  x += step;
  while (x >= s.w) {
    x -= s.w;
    if (++y == s.h) {
      y = 0;
      if (++z == s.d) {
        z = 0;
        ++n;
      }
    }
  }
}

// 8 x 8 transpose of 16-bit values: in[v] holds 8 consecutive columns of
// voxel v (dword i = columns 2i, 2i+1); out[c] holds the 8 voxels of column
// c (dword p = voxels 2p, 2p+1).
__device__ __forceinline__ void transpose8x8(const uint4 (&in)[8], uint4 (&out)[8]) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    uint32_t o[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const uint32_t a = reinterpret_cast<const uint32_t*>(&in[2 * p])[c >> 1];
      const uint32_t b = reinterpret_cast<const uint32_t*>(&in[2 * p + 1])[c >> 1];
      o[p] = (c & 1) ? ((a >> 16) | (b & 0xFFFF0000u)) : ((a & 0xFFFFu) | (b << 16));
    }
    out[c] = make_uint4(o[0], o[1], o[2], o[3]);
  }
}

// Weight gradient tile: TM output channels (32 or 64) x 64 im2col columns,
// reduced over a split's voxels in stages of 64.  A stage of each operand is
// cut into 8-column x 8-voxel blocks; thread t < TM loads dy block t, thread
// TM <= t < TM + 64 loads x block t - TM (8 gathered 16-byte loads, one per
// voxel: the 8 columns share one tap), transposes it in registers and writes
// 8 rows of 16 bytes to LDS ([column][voxel]), the layout the MFMA reduction
// over voxels needs.  With TM = 64 wavefront wv computes rows 16 wv..+15
// against four 16-column tiles; with TM = 32 it computes rows 16 (wv % 2)
// against tiles 2 (wv / 2), +1.  One stage of register prefetch.
template <int TM>
__global__ __launch_bounds__(256) void conv_bwdw_kernel(const uint16_t* __restrict__ x,
                                                        const uint16_t* __restrict__ dy,
                                                        float* __restrict__ part, Shape s, int ci,
                                                        int co, long long chunks_per_split) {
  constexpr int LDW = kWM + kPad;
  __shared__ __attribute__((aligned(16))) uint16_t Ds[TM][LDW];  // [co][m]
  __shared__ __attribute__((aligned(16))) uint16_t Xs[64][LDW];  // [k][m]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K = 27 * ci;
  const int c0 = blockIdx.x * TM;   // co tile
  const int kt0 = blockIdx.y * 64;  // k tile
  const long long mbeg = (long long)blockIdx.z * chunks_per_split * kWM;
  const long long mend = std::min<long long>(s.m, mbeg + chunks_per_split * kWM);

  // this thread's block: columns 8 cb .. 8 cb + 7 of dy (is_dy) or of im2col(x),
  // voxels 8 vb .. 8 vb + 7 of the stage
  const bool is_dy = tid < TM;
  const bool has_block = tid < TM + 64;
  const int blk = is_dy ? tid : tid - TM;
  const int cb = blk >> 3, vb = blk & 7;
  const int col = is_dy ? c0 + 8 * cb : kt0 + 8 * cb;
  const bool col_ok = has_block && (is_dy ? col < co : col < K);
  const int tap = (!is_dy && col_ok) ? col / ci : 0;
  const int ch = is_dy ? 0 : col - tap * ci;
  const int dz = tap / 9 - 1, dyo = (tap / 3) % 3 - 1, dxo = tap % 3 - 1;
  int vn = 0, vz = 0, vy = 0, vx = 0;  // coordinates of the block's first voxel
  {
    const long long m = mbeg + 8 * vb;
    if (m < s.m) unflatten(m, s, vn, vz, vy, vx);
  }
  uint4 raw[8];
  auto gload = [&](long long mc) {
    int n = vn, z = vz, y = vy, xx = vx;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const long long m = mc + 8 * vb + j;
      raw[j] = make_uint4(0, 0, 0, 0);
      if (col_ok && m < mend) {
        if (is_dy) {
          raw[j] = *reinterpret_cast<const uint4*>(dy + m * co + col);
        } else {
          int zz = z + dz, yy = y + dyo, xq = xx + dxo;
          zz = zz < 0 ? zz + s.d : (zz >= s.d ? zz - s.d : zz);
          yy = yy < 0 ? yy + s.h : (yy >= s.h ? yy - s.h : yy);
          xq = xq < 0 ? xq + s.w : (xq >= s.w ? xq - s.w : xq);
          const long long v = (((long long)n * s.d + zz) * s.h + yy) * s.w + xq;
          raw[j] = *reinterpret_cast<const uint4*>(x + v * ci + ch);
        }
      }
      advance_voxel(n, z, y, xx, 1, s);
    }
  };
  constexpr int NT = TM == 64 ? 4 : 2;  // column tiles per wavefront
  const int row0 = TM == 64 ? 16 * wv : 16 * (wv & 1);
  const int tile0 = TM == 64 ? 0 : 2 * (wv >> 1);
  f32x4 acc[NT];
#pragma unroll
  for (int b = 0; b < NT; ++b) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (has_block) gload(mbeg);
  for (long long mc = mbeg; mc < mend; mc += kWM) {
    if (has_block) {
      uint4 tr[8];
      transpose8x8(raw, tr);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        uint16_t* dst = is_dy ? &Ds[8 * cb + e][8 * vb] : &Xs[8 * cb + e][8 * vb];
        *reinterpret_cast<uint4*>(dst) = tr[e];
      }
    }
    __syncthreads();
    if (has_block && mc + kWM < mend) {
      advance_voxel(vn, vz, vy, vx, kWM, s);
      gload(mc + kWM);
    }
    if (c0 + row0 < co) {
#pragma unroll
      for (int ks = 0; ks < kWM; ks += 32) {
        const int kk = ks + 8 * (lane >> 4);
        const bf16x8 a = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const uint4*>(&Ds[row0 + (lane & 15)][kk]));
#pragma unroll
        for (int b = 0; b < NT; ++b) {
          const bf16x8 bf = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const uint4*>(&Xs[(tile0 + b) * 16 + (lane & 15)][kk]));
          acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bf, acc[b], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  float* out = part + (long long)blockIdx.z * co * K;
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    const int k = kt0 + (tile0 + b) * 16 + (lane & 15);
    if (k >= K) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = c0 + row0 + (lane >> 4) * 4 + i;
      if (o < co) out[(long long)o * K + k] = acc[b][i];
    }
  }
}

__global__ void fold_splits_kernel(const float* __restrict__ part, float* __restrict__ dw,
                                   long long n, int splits) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    float a = 0.f;
#pragma unroll 8
    for (int s = 0; s < splits; ++s) a += part[(long long)s * n + i];
    dw[i] = a;
  }
}

// db[c] = sum_m dy[m][c], first pass: block b sums voxels [b per, (b+1) per)
// into part[b][c].  Thread (g, ch) of the G = 256 / c groups handles
// channel ch (consecutive threads read consecutive channels of a voxel) and
// voxels g, g + G, ...; the groups are folded in a fixed order in LDS, and
// fold_splits_kernel sums the blocks in order (deterministic).
__global__ __launch_bounds__(256) void bias_grad_part_kernel(const float* __restrict__ dy,
                                                             float* __restrict__ part,
                                                             long long m, int c,
                                                             long long per) {
  __shared__ float sh[256];
  const int G = c <= 256 ? 256 / c : 1;
  const long long beg = (long long)blockIdx.x * per;
  const long long end = beg + per < m ? beg + per : m;
  for (int cb = 0; cb < c; cb += 256) {
    const int tid = threadIdx.x;
    const int g = c <= 256 ? tid / c : 0;
    const int ch = c <= 256 ? tid % c : cb + tid;
    float a = 0.f;
    if (g < G && ch < c)
      for (long long v = beg + g; v < end; v += G) a += dy[v * c + ch];
    sh[tid] = a;
    __syncthreads();
    if (c <= 256) {
      if (tid < c) {
        float t = 0.f;
        for (int q = 0; q < G; ++q) t += sh[q * c + tid];
        part[(long long)blockIdx.x * c + tid] = t;
      }
    } else if (ch < c) {
      part[(long long)blockIdx.x * c + ch] = a;
    }
    __syncthreads();
    if (c <= 256) break;
  }
}

constexpr int kBiasSplits = 512;

// Bias-gradient partial sums with four consecutive channels per thread (c a
// multiple of 4, at most 1024): thread (g, q) of a block sums channels
// 4q..4q+3 over the block's voxels v = beg + g, beg + g + G, ... (G = 256 /
// (c / 4) voxel groups), then the block adds the G partial sums in order.
// Both nn_bias_grad (dz given, FUSED false) and nn_relu_backward_bias (dz =
// relu'(a) da, stored as BF16, FUSED true) sum in this order, so their db
// agree bit for bit.  vec selects 16-byte FP32 and 8-byte BF16 accesses when
// the pointers allow them (the order is the same either way).  Against one
// channel per thread with 4-byte loads, whose 512 workgroups waited on each
// load in turn: 158 -> 73 us for the largest layer of a 64^3 x 4 training
// step (81 -> 35 us on average).
template <bool FUSED>
__global__ __launch_bounds__(256) void bias4_part_kernel(const float* __restrict__ da,
                                                         const uint16_t* __restrict__ a,
                                                         uint16_t* __restrict__ dzb,
                                                         float* __restrict__ part, long long m,
                                                         int c, long long per, int relu, int vec) {
  __shared__ float4 sh[256];
  const int c4 = c >> 2;
  const int G = 256 / c4;
  const int tid = threadIdx.x, g = tid / c4, q = tid - g * c4;
  const long long beg = (long long)blockIdx.x * per;
  const long long end = beg + per < m ? beg + per : m;
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
  if (g < G) {
#pragma unroll 4
    for (long long v = beg + g; v < end; v += G) {
      const long long i = v * c + 4 * q;
      float z[4];
      if (vec) {
        const float4 t = *reinterpret_cast<const float4*>(da + i);
        z[0] = t.x;
        z[1] = t.y;
        z[2] = t.z;
        z[3] = t.w;
      } else {
        for (int j = 0; j < 4; ++j) z[j] = da[i + j];
      }
      if constexpr (FUSED) {
        if (relu) {
          uint16_t h[4];
          if (vec) {
            const uint2 w = *reinterpret_cast<const uint2*>(a + i);
            h[0] = (uint16_t)w.x;
            h[1] = (uint16_t)(w.x >> 16);
            h[2] = (uint16_t)w.y;
            h[3] = (uint16_t)(w.y >> 16);
          } else {
            for (int j = 0; j < 4; ++j) h[j] = a[i + j];
          }
          for (int j = 0; j < 4; ++j)
            if (!(bf2f(h[j]) > 0.f)) z[j] = 0.f;
        }
        uint16_t o[4];
        for (int j = 0; j < 4; ++j) o[j] = f2bf(z[j]);
        if (vec)
          *reinterpret_cast<uint2*>(dzb + i) =
              make_uint2((uint32_t)o[0] | ((uint32_t)o[1] << 16), (uint32_t)o[2] | ((uint32_t)o[3] << 16));
        else
          for (int j = 0; j < 4; ++j) dzb[i + j] = o[j];
      }
      s.x += z[0];
      s.y += z[1];
      s.z += z[2];
      s.w += z[3];
    }
  }
  sh[tid] = s;
  __syncthreads();
  if (tid < c4) {
    float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int r = 0; r < G; ++r) {
      const float4 u = sh[r * c4 + tid];
      t.x += u.x;
      t.y += u.y;
      t.z += u.z;
      t.w += u.w;
    }
    float* out = part + (long long)blockIdx.x * c + 4 * tid;
    out[0] = t.x;
    out[1] = t.y;
    out[2] = t.z;
    out[3] = t.w;
  }
}
bool bias4(int c) { return c % 4 == 0 && c <= 1024; }

// The backward of a layer's activation, fused with what the convolution's
// backward needs from it: dz = (relu ? (a > 0 ? da : 0) : da) stored as BF16
// (the MFMA operand of both convolution gradients), and the first pass of
// db = sum_m dz[m][c] over the FP32 dz, in bias_grad_part_kernel's order (so
// db is bit-identical to nn_bias_grad of the FP32 dz).
__global__ __launch_bounds__(256) void relu_bwd_bias_part_kernel(
    const float* __restrict__ da, const uint16_t* __restrict__ a, uint16_t* __restrict__ dzb,
    float* __restrict__ part, long long m, int c, long long per, int relu) {
  __shared__ float sh[256];
  const int G = c <= 256 ? 256 / c : 1;
  const long long beg = (long long)blockIdx.x * per;
  const long long end = beg + per < m ? beg + per : m;
  for (int cb = 0; cb < c; cb += 256) {
    const int tid = threadIdx.x;
    const int g = c <= 256 ? tid / c : 0;
    const int ch = c <= 256 ? tid % c : cb + tid;
    float s = 0.f;
    if (g < G && ch < c)
      for (long long v = beg + g; v < end; v += G) {
        const long long i = v * c + ch;
        float z = da[i];
        if (relu && !(bf2f(a[i]) > 0.f)) z = 0.f;
        dzb[i] = f2bf(z);
        s += z;
      }
    sh[tid] = s;
    __syncthreads();
    if (c <= 256) {
      if (tid < c) {
        float t = 0.f;
        for (int q = 0; q < G; ++q) t += sh[q * c + tid];
        part[(long long)blockIdx.x * c + tid] = t;
      }
    } else if (ch < c) {
      part[(long long)blockIdx.x * c + ch] = s;
    }
    __syncthreads();
    if (c <= 256) break;
  }
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

// Four-element forms of the activation, its gradient and the cast (16-byte
// FP32 words, 8-byte BF16 words), for counts that are multiples of 4 and
// aligned pointers.
__device__ __forceinline__ uint2 pack_bf16x4(float a, float b, float c, float d) {
  return make_uint2((uint32_t)f2bf(a) | ((uint32_t)f2bf(b) << 16),
                    (uint32_t)f2bf(c) | ((uint32_t)f2bf(d) << 16));
}

__global__ void relu_fwd_vec_kernel(const float4* __restrict__ z, uint2* __restrict__ a,
                                    long long n4, int relu) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n4;
       i += (long long)gridDim.x * blockDim.x) {
    float4 v = z[i];
    if (relu) {
      v.x = fmaxf(v.x, 0.f);
      v.y = fmaxf(v.y, 0.f);
      v.z = fmaxf(v.z, 0.f);
      v.w = fmaxf(v.w, 0.f);
    }
    a[i] = pack_bf16x4(v.x, v.y, v.z, v.w);
  }
}

__global__ void relu_bwd_vec_kernel(const float4* __restrict__ da, const uint2* __restrict__ a,
                                    float4* __restrict__ dz, long long n4) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n4;
       i += (long long)gridDim.x * blockDim.x) {
    const float4 g = da[i];
    const uint2 h = a[i];
    dz[i] = make_float4(bf2f((uint16_t)h.x) > 0.f ? g.x : 0.f,
                        bf2f((uint16_t)(h.x >> 16)) > 0.f ? g.y : 0.f,
                        bf2f((uint16_t)h.y) > 0.f ? g.z : 0.f,
                        bf2f((uint16_t)(h.y >> 16)) > 0.f ? g.w : 0.f);
  }
}

__global__ void cast_bf16_vec_kernel(const float4* __restrict__ x, uint2* __restrict__ y,
                                     long long n4) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n4;
       i += (long long)gridDim.x * blockDim.x) {
    const float4 v = x[i];
    y[i] = pack_bf16x4(v.x, v.y, v.z, v.w);
  }
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

// Granule forms of the pooling, upsampling, concatenation and split kernels:
// one thread moves 8 BF16 (or 4 FP32) channels of a voxel as one 16-byte
// word, with 32-bit index arithmetic.  Used when the channel counts are
// multiples of the granule, the pointers 16-byte aligned and the element
// count below 2^31; the element forms above cover the rest.
bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

__device__ __forceinline__ void voxel_of(int v, int d, int h, int w, int& n, int& z, int& y,
                                         int& x) {
  x = v % w;
  v /= w;
  y = v % h;
  v /= h;
  z = v % d;
  n = v / d;
}

__global__ void pool_fwd_vec_kernel(const uint4* __restrict__ x, uint4* __restrict__ y, int n_,
                                    int d, int h, int w, int g) {
  const int qd = d / 2, qh = h / 2, qw = w / 2;
  const int total = n_ * qd * qh * qw * g;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int gi = i % g;
    int vn, vz, vy, vx;
    voxel_of(i / g, qd, qh, qw, vn, vz, vy, vx);
    float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int o = 0; o < 8; ++o) {
      const int f = ((vn * d + 2 * vz + (o >> 2)) * h + 2 * vy + ((o >> 1) & 1)) * w + 2 * vx + (o & 1);
      const uint4 u = x[f * g + gi];
      const uint32_t q[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        a[2 * k] += bf2f((uint16_t)q[k]);
        a[2 * k + 1] += bf2f((uint16_t)(q[k] >> 16));
      }
    }
    uint32_t r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      r[k] = (uint32_t)f2bf(0.125f * a[2 * k]) | ((uint32_t)f2bf(0.125f * a[2 * k + 1]) << 16);
    y[i] = make_uint4(r[0], r[1], r[2], r[3]);
  }
}

__global__ void pool_bwd_vec_kernel(const float4* __restrict__ dy, float4* __restrict__ dx,
                                    int n_, int d, int h, int w, int g) {
  const int total = n_ * d * h * w * g;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int gi = i % g;
    int vn, vz, vy, vx;
    voxel_of(i / g, d, h, w, vn, vz, vy, vx);
    const int p = ((vn * (d / 2) + vz / 2) * (h / 2) + vy / 2) * (w / 2) + vx / 2;
    const float4 v = dy[p * g + gi];
    dx[i] = make_float4(0.125f * v.x, 0.125f * v.y, 0.125f * v.z, 0.125f * v.w);
  }
}

// coarse (n, d, h, w) -> fine (n, 2d, 2h, 2w)
__global__ void up_fwd_vec_kernel(const uint4* __restrict__ x, uint4* __restrict__ y, int n_,
                                  int d, int h, int w, int g) {
  const int total = n_ * 8 * d * h * w * g;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int gi = i % g;
    int vn, vz, vy, vx;
    voxel_of(i / g, 2 * d, 2 * h, 2 * w, vn, vz, vy, vx);
    const int p = ((vn * d + vz / 2) * h + vy / 2) * w + vx / 2;
    y[i] = x[p * g + gi];
  }
}

__global__ void up_bwd_vec_kernel(const float4* __restrict__ dy, float4* __restrict__ dx, int n_,
                                  int d, int h, int w, int g) {
  const int total = n_ * d * h * w * g;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int gi = i % g;
    int vn, vz, vy, vx;
    voxel_of(i / g, d, h, w, vn, vz, vy, vx);
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int o = 0; o < 8; ++o) {
      const int f = ((vn * 2 * d + 2 * vz + (o >> 2)) * 2 * h + 2 * vy + ((o >> 1) & 1)) * 2 * w +
                    2 * vx + (o & 1);
      const float4 v = dy[f * g + gi];
      a.x += v.x;
      a.y += v.y;
      a.z += v.z;
      a.w += v.w;
    }
    dx[i] = a;
  }
}

// granules of 8 bf16 channels: ga + gb per voxel
__global__ void concat_vec_kernel(const uint4* __restrict__ a, const uint4* __restrict__ b,
                                  uint4* __restrict__ y, int m, int ga, int gb) {
  const int g = ga + gb, total = m * g;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int v = i / g, k = i % g;
    y[i] = k < ga ? a[v * ga + k] : b[v * gb + k - ga];
  }
}

// granules of 4 fp32 channels
__global__ void split_vec_kernel(const float4* __restrict__ dy, float4* __restrict__ da,
                                 float4* __restrict__ db, int m, int ga, int gb) {
  const int g = ga + gb, total = m * g;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int v = i / g, k = i % g;
    if (k < ga) {
      if (da) da[v * ga + k] = dy[i];
    } else if (db) {
      db[v * gb + k - ga] = dy[i];
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ C ABI

namespace {

template <bool ACT>
lbm_status conv_forward(const void* x, const void* w, const float* bias, void* y, int n, int d,
                        int h, int wd, int ci, int co, int relu, void* stream) {
  if (!x || !w || !y || bad_shape(n, d, h, wd) || ci < 8 || ci % 8 || co < 1)
    return LBM_ERR_INVALID_ARG;
  const Shape s = shape_of(n, d, h, wd);
  if (s.m >= (1LL << 31)) return LBM_ERR_INVALID_ARG;  // voxel indices are 32-bit in the tables
  const int bn = co <= 16 ? 16 : (co <= 32 ? 32 : 64);
  const hipStream_t st = (hipStream_t)stream;
  const uint16_t* xx = (const uint16_t*)x;
  const uint16_t* ww = (const uint16_t*)w;
  // spatial tiles where the box and channels allow and the grid is not tiny
  const long long tiles = s.m / (kTZ * kTY * kTX);
  if (ci % kCC == 0 && d % kTZ == 0 && h % kTY == 0 && wd % kTX == 0 &&
      tiles * ((co + bn - 1) / bn) >= 128) {
    dim3 sgrid((unsigned)tiles, (unsigned)((co + bn - 1) / bn));
    if (bn == 16)
      conv_fwd_spatial_kernel<16, ACT><<<sgrid, 256, 0, st>>>(xx, ww, bias, y, s, ci, co, relu);
    else if (bn == 32)
      conv_fwd_spatial_kernel<32, ACT><<<sgrid, 256, 0, st>>>(xx, ww, bias, y, s, ci, co, relu);
    else
      conv_fwd_spatial_kernel<64, ACT><<<sgrid, 256, 0, st>>>(xx, ww, bias, y, s, ci, co, relu);
    return check_launch();
  }
  dim3 grid((unsigned)((s.m + 127) / 128), (unsigned)((co + bn - 1) / bn));
  if (bn == 16)
    conv_fwd_tiled_kernel<16, ACT><<<grid, 256, 0, st>>>(xx, ww, bias, y, s, ci, co, relu);
  else if (bn == 32)
    conv_fwd_tiled_kernel<32, ACT><<<grid, 256, 0, st>>>(xx, ww, bias, y, s, ci, co, relu);
  else
    conv_fwd_tiled_kernel<64, ACT><<<grid, 256, 0, st>>>(xx, ww, bias, y, s, ci, co, relu);
  return check_launch();
}

}  // namespace

NN_API lbm_status nn_conv3d_forward(const void* x, const void* w, const float* bias, float* y,
                                    int n, int d, int h, int wd, int ci, int co, void* stream) {
  return conv_forward<false>(x, w, bias, y, n, d, h, wd, ci, co, 0, stream);
}

NN_API lbm_status nn_conv3d_forward_act(const void* x, const void* w, const float* bias, void* a,
                                        int n, int d, int h, int wd, int ci, int co, int relu,
                                        void* stream) {
  if (relu != 0 && relu != 1) return LBM_ERR_INVALID_ARG;
  return conv_forward<true>(x, w, bias, a, n, d, h, wd, ci, co, relu, stream);
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

// The spatially tiled weight gradient applies (and with how many splits).
static bool bwdw_spatial(int n, int d, int h, int wd, int ci, int co, int* splits) {
  const long long tiles = (long long)n * d * h * wd / (kTZ * kTY * kTX);
  if (d % kTZ || h % kTY || wd % kTX || tiles < 256) return false;
  // about 512 blocks over the channel tiles, at least two voxel tiles each
  const int ct = ci % 32 == 0 ? 32 : 16, rt = co % 32 == 0 ? 32 : 16;
  const long long chan_tiles = (long long)((ci + ct - 1) / ct) * ((co + rt - 1) / rt);
  *splits = (int)std::max<long long>(
      1, std::min<long long>({256, tiles / 2, 512 / std::max<long long>(chan_tiles, 1)}));
  return true;
}

NN_API lbm_status nn_conv3d_backward_weight_workspace(int n, int d, int h, int wd, int ci, int co,
                                                      size_t* bytes, int* splits) {
  if (!bytes || bad_shape(n, d, h, wd) || ci < 8 || ci % 8 || co < 8 || co % 8)
    return LBM_ERR_INVALID_ARG;
  int ssp = 0;
  if (bwdw_spatial(n, d, h, wd, ci, co, &ssp)) {
    *bytes = (size_t)ssp * co * 27 * ci * sizeof(float);
    if (splits) *splits = ssp;
    return LBM_OK;
  }
  const long long m = (long long)n * d * h * wd;
  const int tm = co <= 32 ? 32 : 64;
  const long long tiles = (long long)((co + tm - 1) / tm) * ((27 * ci + 63) / 64);
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
  const long long nw = (long long)co * 27 * ci;
  int ssp = 0;
  if (bwdw_spatial(n, d, h, wd, ci, co, &ssp)) {
    const int tiles = (int)(s.m / (kTZ * kTY * kTX));
    // channel tiles: 32 where the count is a multiple of 32, else 16 (zero padded)
    const int ct = ci % 32 == 0 ? 2 : 1, rt = co % 32 == 0 ? 2 : 1;
    dim3 sgrid((unsigned)ssp, (unsigned)((ci + 16 * ct - 1) / (16 * ct)),
               (unsigned)((co + 16 * rt - 1) / (16 * rt)));
    const uint16_t* xx = (const uint16_t*)x;
    const uint16_t* dd = (const uint16_t*)dy;
    float* pp = (float*)ws;
    const hipStream_t st = (hipStream_t)stream;
    if (rt == 2 && ct == 2)
      conv_bwdw_spatial_kernel<2, 2><<<sgrid, 256, 0, st>>>(xx, dd, pp, s, ci, co, tiles);
    else if (rt == 2)
      conv_bwdw_spatial_kernel<2, 1><<<sgrid, 256, 0, st>>>(xx, dd, pp, s, ci, co, tiles);
    else if (ct == 2)
      conv_bwdw_spatial_kernel<1, 2><<<sgrid, 256, 0, st>>>(xx, dd, pp, s, ci, co, tiles);
    else
      conv_bwdw_spatial_kernel<1, 1><<<sgrid, 256, 0, st>>>(xx, dd, pp, s, ci, co, tiles);
    fold_splits_kernel<<<grid_for(nw), 256, 0, (hipStream_t)stream>>>((const float*)ws, dw, nw,
                                                                       ssp);
    return check_launch();
  }
  const long long chunks = (s.m + kWM - 1) / kWM;
  const long long per = (chunks + sp - 1) / sp;
  const int tm = co <= 32 ? 32 : 64;
  dim3 grid((unsigned)((co + tm - 1) / tm), (unsigned)((27 * ci + 63) / 64), (unsigned)sp);
  if (tm == 32)
    conv_bwdw_kernel<32><<<grid, 256, 0, (hipStream_t)stream>>>(
        (const uint16_t*)x, (const uint16_t*)dy, (float*)ws, s, ci, co, per);
  else
    conv_bwdw_kernel<64><<<grid, 256, 0, (hipStream_t)stream>>>(
        (const uint16_t*)x, (const uint16_t*)dy, (float*)ws, s, ci, co, per);
  fold_splits_kernel<<<grid_for(nw), 256, 0, (hipStream_t)stream>>>((const float*)ws, dw, nw, sp);
  return check_launch();
}

NN_API lbm_status nn_bias_grad_workspace(long long m, int c, size_t* bytes) {
  if (!bytes || m < 1 || c < 1) return LBM_ERR_INVALID_ARG;
  const long long splits = std::min<long long>(kBiasSplits, (m + 255) / 256);
  *bytes = (size_t)splits * c * sizeof(float);
  return LBM_OK;
}

NN_API lbm_status nn_bias_grad(const float* dy, float* db, void* ws, size_t ws_bytes, long long m,
                               int c, void* stream) {
  size_t need = 0;
  lbm_status st = nn_bias_grad_workspace(m, c, &need);
  if (st != LBM_OK || !dy || !db) return LBM_ERR_INVALID_ARG;
  if (!ws || ws_bytes < need) return LBM_ERR_WORKSPACE;
  const long long splits = need / ((size_t)c * sizeof(float));
  const long long per = (m + splits - 1) / splits;
  if (bias4(c))
    bias4_part_kernel<false><<<(unsigned)splits, 256, 0, (hipStream_t)stream>>>(
        dy, nullptr, nullptr, (float*)ws, m, c, per, 0, aligned16(dy) ? 1 : 0);
  else
    bias_grad_part_kernel<<<(unsigned)splits, 256, 0, (hipStream_t)stream>>>(dy, (float*)ws, m,
                                                                            c, per);
  fold_splits_kernel<<<grid_for(c), 256, 0, (hipStream_t)stream>>>((const float*)ws, db, c,
                                                                  (int)splits);
  return check_launch();
}

NN_API lbm_status nn_relu_backward_bias(const float* da, const void* a, void* dz, float* db,
                                       void* ws, size_t ws_bytes, long long m, int c, int relu,
                                       void* stream) {
  size_t need = 0;
  lbm_status st = nn_bias_grad_workspace(m, c, &need);
  if (st != LBM_OK || !da || !dz || !db || (relu != 0 && relu != 1) || (relu && !a))
    return LBM_ERR_INVALID_ARG;
  if (!ws || ws_bytes < need) return LBM_ERR_WORKSPACE;
  const long long splits = need / ((size_t)c * sizeof(float));
  const long long per = (m + splits - 1) / splits;
  if (bias4(c)) {
    const bool vec = aligned16(da) && ((uintptr_t)dz & 7) == 0 && (!relu || ((uintptr_t)a & 7) == 0);
    bias4_part_kernel<true><<<(unsigned)splits, 256, 0, (hipStream_t)stream>>>(
        da, (const uint16_t*)a, (uint16_t*)dz, (float*)ws, m, c, per, relu, vec ? 1 : 0);
  } else {
    relu_bwd_bias_part_kernel<<<(unsigned)splits, 256, 0, (hipStream_t)stream>>>(
        da, (const uint16_t*)a, (uint16_t*)dz, (float*)ws, m, c, per, relu);
  }
  fold_splits_kernel<<<grid_for(c), 256, 0, (hipStream_t)stream>>>((const float*)ws, db, c,
                                                                  (int)splits);
  return check_launch();
}

NN_API lbm_status nn_activation_forward(const float* z, void* a, long long n, int relu,
                                        void* stream) {
  if (!z || !a || n < 0) return LBM_ERR_INVALID_ARG;
  if (n % 4 == 0 && aligned16(z) && ((uintptr_t)a & 7) == 0) {
    relu_fwd_vec_kernel<<<grid_for(n / 4), 256, 0, (hipStream_t)stream>>>(
        (const float4*)z, (uint2*)a, n / 4, relu);
    return check_launch();
  }
  relu_fwd_kernel<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(z, (uint16_t*)a, n, relu);
  return check_launch();
}

NN_API lbm_status nn_relu_backward(const float* da, const void* a, float* dz, long long n,
                                   void* stream) {
  if (!da || !a || !dz || n < 0) return LBM_ERR_INVALID_ARG;
  if (n % 4 == 0 && aligned16(da) && aligned16(dz) && ((uintptr_t)a & 7) == 0) {
    relu_bwd_vec_kernel<<<grid_for(n / 4), 256, 0, (hipStream_t)stream>>>(
        (const float4*)da, (const uint2*)a, (float4*)dz, n / 4);
    return check_launch();
  }
  relu_bwd_kernel<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(da, (const uint16_t*)a, dz, n);
  return check_launch();
}

NN_API lbm_status nn_cast_bf16(const float* x, void* y, long long n, void* stream) {
  if (!x || !y || n < 0) return LBM_ERR_INVALID_ARG;
  if (n % 4 == 0 && aligned16(x) && ((uintptr_t)y & 7) == 0) {
    cast_bf16_vec_kernel<<<grid_for(n / 4), 256, 0, (hipStream_t)stream>>>(
        (const float4*)x, (uint2*)y, n / 4);
    return check_launch();
  }
  cast_bf16_kernel<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(x, (uint16_t*)y, n);
  return check_launch();
}

NN_API lbm_status nn_pool2_forward(const void* x, void* y, int n, int d, int h, int w, int c,
                                   void* stream) {
  if (!x || !y || bad_shape(n, d, h, w) || d % 2 || h % 2 || w % 2 || c < 1)
    return LBM_ERR_INVALID_ARG;
  const Shape s = shape_of(n, d, h, w);
  if (c % 8 == 0 && aligned16(x) && aligned16(y) && s.m * c < (1LL << 31)) {
    pool_fwd_vec_kernel<<<grid_for(s.m / 8 * (c / 8)), 256, 0, (hipStream_t)stream>>>(
        (const uint4*)x, (uint4*)y, n, d, h, w, c / 8);
    return check_launch();
  }
  pool_fwd_kernel<<<grid_for(s.m / 8 * c), 256, 0, (hipStream_t)stream>>>(
      (const uint16_t*)x, (uint16_t*)y, s, c);
  return check_launch();
}

NN_API lbm_status nn_pool2_backward(const float* dy, float* dx, int n, int d, int h, int w, int c,
                                    void* stream) {
  if (!dy || !dx || bad_shape(n, d, h, w) || d % 2 || h % 2 || w % 2 || c < 1)
    return LBM_ERR_INVALID_ARG;
  const Shape s = shape_of(n, d, h, w);
  if (c % 4 == 0 && aligned16(dy) && aligned16(dx) && s.m * c < (1LL << 31)) {
    pool_bwd_vec_kernel<<<grid_for(s.m * (c / 4)), 256, 0, (hipStream_t)stream>>>(
        (const float4*)dy, (float4*)dx, n, d, h, w, c / 4);
    return check_launch();
  }
  pool_bwd_kernel<<<grid_for(s.m * c), 256, 0, (hipStream_t)stream>>>(dy, dx, s, c);
  return check_launch();
}

// Periodic trilinear prolongation by 2 (the two-grid warm start): fine node
// i of an axis sits between coarse nodes, 3/4 from the nearer one m = i / 2
// and 1/4 from the farther (m - 1 for even i, m + 1 for odd i), so it takes
// 0.75 x[m] + 0.25 x[far].  The three axes are applied in the order z, y, x,
// then the channel scale.
__global__ void prolong2_kernel(const float* __restrict__ x, float* __restrict__ y, int n, int d,
                                int h, int w, int cx, int c, const float* __restrict__ scale,
                                long long total) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c);
    long long r = i / c;
    const int X = (int)(r % (2 * w));
    r /= 2 * w;
    const int Y = (int)(r % (2 * h));
    r /= 2 * h;
    const int Z = (int)(r % (2 * d));
    const int b = (int)(r / (2 * d));
    const int xn = X >> 1, yn = Y >> 1, zn = Z >> 1;
    const int xf = (X & 1) ? (xn + 1 == w ? 0 : xn + 1) : (xn == 0 ? w - 1 : xn - 1);
    const int yf = (Y & 1) ? (yn + 1 == h ? 0 : yn + 1) : (yn == 0 ? h - 1 : yn - 1);
    const int zf = (Z & 1) ? (zn + 1 == d ? 0 : zn + 1) : (zn == 0 ? d - 1 : zn - 1);
    auto at = [&](int zz, int yy, int xx) {
      return x[((((long long)b * d + zz) * h + yy) * w + xx) * cx + ch];
    };
    float a[2];  // the y-then-z interpolated values at the near and far x
    for (int q = 0; q < 2; ++q) {
      const int xx = q ? xf : xn;
      const float bn = 0.75f * at(zn, yn, xx) + 0.25f * at(zf, yn, xx);
      const float bf = 0.75f * at(zn, yf, xx) + 0.25f * at(zf, yf, xx);
      a[q] = 0.75f * bn + 0.25f * bf;
    }
    const float v = 0.75f * a[0] + 0.25f * a[1];
    y[i] = scale ? v * scale[ch] : v;
  }
}

NN_API lbm_status nn_prolongate2(const float* x, float* y, int n, int d, int h, int w, int cx,
                                 int c, const float* scale, void* stream) {
  if (!x || !y || bad_shape(n, d, h, w) || cx < 1 || c < 1 || c > cx)
    return LBM_ERR_INVALID_ARG;
  const long long total = 8LL * n * d * h * w * c;
  prolong2_kernel<<<grid_for(total), 256, 0, (hipStream_t)stream>>>(x, y, n, d, h, w, cx, c, scale,
                                                                    total);
  return check_launch();
}

// Start fields of a warm start, for lbm_init_equilibrium_device, from
// predicted targets t (n boxes of d x h x w, cx channels; velocity targets in
// channels 0-2) and the fluid mask: drho = -(delta_rho / w)(x - (w - 1)/2) on
// fluid cells (the linear profile of the pressure drop), u = factor * t on
// fluid cells none of whose 18 lattice neighbours (periodic in the box) is
// solid, 0 elsewhere.  fields: [drho | u_x | u_y | u_z], n d h w values each.
__global__ void warm_fields_kernel(const float* __restrict__ t, int cx,
                                   const uint8_t* __restrict__ fluid, double* __restrict__ fields,
                                   int n, int d, int h, int w, double factor, double delta_rho) {
  const long long total = (long long)n * d * h * w;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % w);
    long long r = i / w;
    const int y = (int)(r % h);
    r /= h;
    const int z = (int)(r % d);
    const long long box = (r / d) * (long long)d * h * w;
    const bool f = fluid[i] != 0;
    bool wall = false;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int a = (dz != 0) + (dy != 0) + (dx != 0);
          if (a == 0 || a == 3) continue;  // the 18 moving D3Q19 directions
          const int zz = (z + dz + d) % d, yy = (y + dy + h) % h, xx = (x + dx + w) % w;
          wall |= fluid[box + ((long long)zz * h + yy) * w + xx] == 0;
        }
    const double xc = x - (w - 1) / 2.0;
    fields[i] = f ? -(delta_rho / w) * xc : 0.0;
    for (int k = 0; k < 3; ++k)
      fields[(1 + k) * total + i] = (f && !wall) ? (double)t[i * cx + k] * factor : 0.0;
  }
}

NN_API lbm_status nn_warm_start_fields(const float* t, int cx, const void* fluid, double* fields,
                                       int n, int d, int h, int w, double factor,
                                       double delta_rho, void* stream) {
  if (!t || !fluid || !fields || bad_shape(n, d, h, w) || cx < 3) return LBM_ERR_INVALID_ARG;
  const long long total = (long long)n * d * h * w;
  warm_fields_kernel<<<grid_for(total), 256, 0, (hipStream_t)stream>>>(
      t, cx, (const uint8_t*)fluid, fields, n, d, h, w, factor, delta_rho);
  return check_launch();
}

NN_API lbm_status nn_upsample2_forward(const void* x, void* y, int n, int d, int h, int w, int c,
                                       void* stream) {
  if (!x || !y || bad_shape(n, d, h, w) || c < 1) return LBM_ERR_INVALID_ARG;
  const Shape q = shape_of(n, d, h, w);
  if (c % 8 == 0 && aligned16(x) && aligned16(y) && q.m * 8 * c < (1LL << 31)) {
    up_fwd_vec_kernel<<<grid_for(q.m * 8 * (c / 8)), 256, 0, (hipStream_t)stream>>>(
        (const uint4*)x, (uint4*)y, n, d, h, w, c / 8);
    return check_launch();
  }
  up_fwd_kernel<<<grid_for(q.m * 8 * c), 256, 0, (hipStream_t)stream>>>(
      (const uint16_t*)x, (uint16_t*)y, q, c);
  return check_launch();
}

NN_API lbm_status nn_upsample2_backward(const float* dy, float* dx, int n, int d, int h, int w,
                                        int c, void* stream) {
  if (!dy || !dx || bad_shape(n, d, h, w) || c < 1) return LBM_ERR_INVALID_ARG;
  const Shape q = shape_of(n, d, h, w);
  if (c % 4 == 0 && aligned16(dy) && aligned16(dx) && q.m * 8 * c < (1LL << 31)) {
    up_bwd_vec_kernel<<<grid_for(q.m * (c / 4)), 256, 0, (hipStream_t)stream>>>(
        (const float4*)dy, (float4*)dx, n, d, h, w, c / 4);
    return check_launch();
  }
  up_bwd_kernel<<<grid_for(q.m * c), 256, 0, (hipStream_t)stream>>>(dy, dx, q, c);
  return check_launch();
}

NN_API lbm_status nn_concat_channels(const void* a, const void* b, void* y, long long m, int ca,
                                     int cb, void* stream) {
  if (!a || !b || !y || m < 1 || ca < 1 || cb < 1) return LBM_ERR_INVALID_ARG;
  if (ca % 8 == 0 && cb % 8 == 0 && aligned16(a) && aligned16(b) && aligned16(y) &&
      m * (ca + cb) < (1LL << 31)) {
    concat_vec_kernel<<<grid_for(m * ((ca + cb) / 8)), 256, 0, (hipStream_t)stream>>>(
        (const uint4*)a, (const uint4*)b, (uint4*)y, (int)m, ca / 8, cb / 8);
    return check_launch();
  }
  concat_kernel<<<grid_for(m * (ca + cb)), 256, 0, (hipStream_t)stream>>>(
      (const uint16_t*)a, (const uint16_t*)b, (uint16_t*)y, m, ca, cb);
  return check_launch();
}

NN_API lbm_status nn_split_channels(const float* dy, float* da, float* db, long long m, int ca,
                                    int cb, void* stream) {
  if (!dy || m < 1 || ca < 1 || cb < 1) return LBM_ERR_INVALID_ARG;
  if (ca % 4 == 0 && cb % 4 == 0 && aligned16(dy) && aligned16(da) && aligned16(db) &&
      m * (ca + cb) < (1LL << 31)) {
    split_vec_kernel<<<grid_for(m * ((ca + cb) / 4)), 256, 0, (hipStream_t)stream>>>(
        (const float4*)dy, (float4*)da, (float4*)db, (int)m, ca / 4, cb / 4);
    return check_launch();
  }
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
