// HIP kernels of the D3Q19 hot path for gfx950 (MI355X).
//
// Data layout in HBM: two population buffers (A: current post-collision
// state, B: next) of g_k = f_k - w_k, 19 values per cell address, stored in
// runs (Tiling::slot): a run of 64 or 128 consecutive addresses holds its 19
// directions one after the other (FP32, FP64), or the whole state is 19
// padded direction planes (16-bit values).  Cells are stored in tiled order
// (Tiling): each z plane is cut into tiles of 64 cells, one wavefront each.
// States well beyond the last-level cache use compact tiles (16 x 4, or
// 32 x 2 for 16-bit values), so a 128-byte line covers a compact patch of
// cells rather than a stretch of one row, and where sphere surfaces cut the
// lines, fewer of them are fetched for a few fluid cells; smaller states use
// 64 x 1 tiles, i.e. plain rows.  A uint8 class per cell says whether the
// cell is solid and whether it has wall links; the uint32 flag word of a
// cell with links marks the directions whose pull source is
// solid.  For such a wall link the otherwise unused slot of the solid source
// node in direction k holds the CLI coefficient a = (1-2q)/(1+2q) (0 for
// fallback links), written once at bind time into both buffers.  In batches,
// solid cells next to fluid cells may copy their link slots and write zeros
// elsewhere (whole-line writes, solid_stores); otherwise solid cells are not
// written, so the slots persist either way.
//
// The step is a pull scheme: each fluid cell gathers its 19 incoming values
// from its neighbours (one read per element of A), applies the wall rule and
// the periodic pressure jump, collides, and writes its 19 values to B (one
// aligned write per element).  It is HBM-bandwidth bound.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lattice.hpp"

namespace lbm {

enum { kSRT = 0, kTRT = 1, kMRT = 2 };
// Wall templates: simple bounce-back, CLI (coefficient a in the solid slot),
// and the general interpolated rules (LIBB, QIBB, IEBB, MR; q in the solid
// slot, rule chosen at run time by StepParams::wall, FP32/FP64 only).
enum { kSBB = 0, kCLI = 1, kGEN = 2 };
// run-time rule numbers (lbm_wall)
enum { kRuleSBB = 0, kRuleCLI = 1, kRuleLIBB = 2, kRuleQIBB = 3, kRuleIEBB = 4, kRuleMR = 5 };

// Tiled cell order.  A z plane of nx x ny cells is padded to whole tiles of
// 2^tw_log2 x 2^th_log2 = 64 cells; tiles follow each other in x, then y;
// cells inside a tile in x, then y; planes follow in z.  The address of
// (x, y, z) splits into independent x, y and z parts, so neighbour addresses
// are sums of three precomputed offsets.  Padding cells are marked solid and
// never read as a neighbour (the periodic wrap uses nx and ny).
struct Tiling {
  int nx, ny;            // box edge in x and y (cells)
  int tw_log2, th_log2;  // tile width and height, log2 (sum 6 or 7: tiles of 64 or 128 cells)
  int ntx;               // tiles per tile row (padded nx / tile width)
  int nty;               // tile rows per plane
  int plane;             // cells per z plane including padding: ntx * nty * tile cells
  int run_log2;          // state buffers: runs of 2^run_log2 consecutive addresses,
  long long run_pitch;   // ... each direction of a run run_pitch elements after the last
  __host__ __device__ int tile_log2() const { return tw_log2 + th_log2; }
  __host__ __device__ int xpart(int x) const {
    return ((x >> tw_log2) << tile_log2()) | (x & ((1 << tw_log2) - 1));
  }
  __host__ __device__ int ypart(int y) const {
    return (y >> th_log2) * (ntx << tile_log2()) + ((y & ((1 << th_log2) - 1)) << tw_log2);
  }
  __host__ __device__ int at(int x, int y, int z) const { return xpart(x) + ypart(y) + z * plane; }
  // inverse of at() (padding cells give x >= nx or y >= ny)
  __host__ __device__ void coords(int a, int& x, int& y, int& z) const {
    z = a / plane;
    const int r = a - z * plane;
    const int t = r >> tile_log2(), l = r & ((1 << tile_log2()) - 1);
    x = ((t % ntx) << tw_log2) + (l & ((1 << tw_log2) - 1));
    y = ((t / ntx) << th_log2) + (l >> tw_log2);
  }
  // Index of direction k of the cell at address a in a state buffer.  The
  // addresses are cut into runs of 2^run_log2 and each run stores its 19
  // directions one after the other, run_pitch apart: with short runs (two
  // tiles, run_pitch = 2^run_log2) a wavefront's 19 loads or stores lie close
  // together; with one run holding all addresses (run_pitch the padded
  // address count) the state is 19 direction planes.
  __host__ __device__ long long slot(int k, long long a) const {
    return ((a >> run_log2) * kQ + k) * run_pitch + (a & ((1LL << run_log2) - 1));
  }
  // address of the cell with row-major index c = x + nx (y + ny z)
  __host__ __device__ int from_linear(long long c) const {
    const int x = (int)(c % nx);
    const long long r = c / nx;
    return at(x, (int)(r % ny), (int)(r / ny));
  }
};

// FP32 and FP64 states are cut into runs of 2^7 addresses for one domain and
// of 2^6 for batches (every batch cell then starts on a run); every z plane
// starts on a run (state_base).
constexpr int kStepRunLog2 = 7, kBatchRunLog2 = 6;

// Tiling::slot for a kernel's storage type, with the layout fixed at compile
// time (16-bit values: direction planes, k * run_pitch + a; FP32 and FP64:
// runs of 2^run_log2 addresses), so that the per-lane address is the cell
// address plus a wavefront-uniform offset where it can be.
template <typename S>
__device__ __forceinline__ long long state_slot(const Tiling& t, int k, long long a) {
  if constexpr (sizeof(S) == 2)
    return k * t.run_pitch + a;
  else
    return ((((a >> t.run_log2) * kQ) + k) << t.run_log2) + (a & ((1LL << t.run_log2) - 1));
}

// Byte offset of direction k of the cell at address zstart + r, split into a
// wavefront-uniform part (direction k and the z plane that starts at address
// zstart, a whole number of runs) and a 32-bit part per lane (the in-plane
// address r), so that a load is a scalar base plus a lane offset.  The host
// keeps planes small enough for the lane part to fit in 32 bits.
// The run length stays a run-time value here: the per-direction bases are
// then computed on the scalar unit and every pull is a scalar base plus a
// lane offset (512^3 sphere pack, FP32: 2.31 ms per step, against 2.37 ms
// with the run length fixed at compile time, where the compiler folds the
// direction offsets into 64-bit lane addresses, and 2.34-2.36 ms with 64-bit
// lane addresses throughout).
template <typename S>
__device__ __forceinline__ long long state_base(const Tiling& t, int k, long long zstart) {
  if constexpr (sizeof(S) == 2)
    return 2LL * (k * t.run_pitch + zstart);
  else  // zstart / run length runs of kQ directions before, then k directions
    return (long long)sizeof(S) * (zstart * kQ + ((long long)k << t.run_log2));
}
template <typename S>
__device__ __forceinline__ uint32_t state_lane(const Tiling& t, int r) {
  if constexpr (sizeof(S) == 2) {
    return 2u * (uint32_t)r;
  } else {
    const uint32_t run = (uint32_t)r >> t.run_log2, in = (uint32_t)r & ((1u << t.run_log2) - 1u);
    return (uint32_t)sizeof(S) * (((run * (uint32_t)kQ) << t.run_log2) + in);
  }
}
template <typename S, typename P>
__device__ __forceinline__ P* state_at(P* base, const Tiling& t, int k, long long zstart, int r) {
  using B = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<B*>(base) + state_base<S>(t, k, zstart) +
                              state_lane<S>(t, r));
}

// Element of direction k of the cell at address a: for direction planes the
// plane's base (wavefront-uniform) plus the 32-bit address.
template <typename S, typename P>
__device__ __forceinline__ P* state_ptr(P* base, const Tiling& t, int k, int a) {
  if constexpr (sizeof(S) == 2)
    return (base + k * t.run_pitch) + a;
  else
    return base + state_slot<S>(t, k, a);
}

// Cell classes (one byte per cell, tiled order).
constexpr uint8_t kClsSolid = 1;  // solid (or padding) cell
constexpr uint8_t kClsLinks = 2;  // the cell's flag word has link bits
constexpr uint8_t kClsNearWall = 4;  // x_f2 of a wall link (IEBB reads its velocity)

struct StepParams {
  Tiling t;
  int nx, ny, nz;
  double jump_axis;   // w_axis * delta_rho
  double jump_diag;   // w_diag * delta_rho
  double omega_p;     // 1/tau (SRT, TRT symmetric, MRT viscous modes)
  double omega_m;     // TRT antisymmetric rate
  double s_e;         // MRT energy modes 1, 2
  double s_zeta;      // MRT remaining kinetic modes
  double sigma;       // 16-bit storage: stored h_k = sigma * g_k / w_k
  float dec[3];       // ... h -> g factors w_k / sigma per weight class (rest, axis, diagonal)
  float enc[3];       // ... g -> h factors sigma / w_k
  // the rates and jumps above rounded to FP32 (the FP32 compute type)
  float omega_pf, omega_mf, s_ef, s_zetaf, jump_axisf, jump_diagf;
  unsigned seed;      // stochastic rounding: per-step seed
  int wall;           // wall rule (lbm_wall) for the general wall template
  int solid_writes;   // batches: which solid cells store (solid_stores): 0, 1, 2
  // single-domain step workgroups: bw x bh wavefronts cover bw units (a tile,
  // or two x-adjacent tiles with two cells per lane) of bh consecutive tile
  // rows; nbx workgroups span a band of bh tile rows
  int bw, bh, nbx;
  // IEBB, one domain: the velocity (momentum j, as stored_moments) of the
  // cells marked kClsNearWall, 4 values of the compute type per address;
  // side_in belongs to the step's source state, side_out to the state it
  // writes (null: IEBB sums the 19 stored values at x_f2 instead)
  void* side_in;
  void* side_out;
};

// ------------------------------------------------------------ storage types
// FP64 and FP32 store g_k directly.  The 16-bit types store h_k = sigma g_k /
// w_k: dividing by the weight puts the 19 directions on one scale and sigma
// (a power of two) moves that scale into the normal range of the format.
// Values are computed in FP32 and rounded to nearest-even on store.

struct bf16_t {
  uint16_t u;
};
using fp16_t = _Float16;

template <typename S>
struct Storage {
  using compute = float;
  static constexpr bool scaled = false;
  __device__ __host__ static float to_float(S v) { return (float)v; }
  __device__ __host__ static S from_float(float v) { return (S)v; }
};
template <>
struct Storage<double> {
  using compute = double;
  static constexpr bool scaled = false;
  __device__ __host__ static double to_float(double v) { return v; }
  __device__ __host__ static double from_float(double v) { return v; }
};
template <>
struct Storage<fp16_t> {
  using compute = float;
  static constexpr bool scaled = true;
  __device__ __host__ static float to_float(fp16_t v) { return (float)v; }
  __device__ __host__ static fp16_t from_float(float v) { return (fp16_t)v; }
};
template <>
struct Storage<bf16_t> {
  using compute = float;
  static constexpr bool scaled = true;
  __device__ __host__ static float to_float(bf16_t v) {
    return __builtin_bit_cast(float, (uint32_t)v.u << 16);
  }
  // round to nearest, ties to even; NaN stays a quiet NaN
  __device__ __host__ static bf16_t from_float(float f) {
    uint32_t b = __builtin_bit_cast(uint32_t, f);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return bf16_t{(uint16_t)((b >> 16) | 0x40u)};
    b += 0x7FFFu + ((b >> 16) & 1u);
    return bf16_t{(uint16_t)(b >> 16)};
  }
};

// Stochastic-rounding variants: the stored value is the 16-bit neighbour
// below or above (in magnitude) with probabilities given by the distance, so
// the rounding error has zero mean.  r is a uniform 32-bit random word.
struct fp16s_t {
  _Float16 v;
};
struct bf16s_t {
  uint16_t u;
};
template <>
struct Storage<fp16s_t> {
  using compute = float;
  static constexpr bool scaled = true;
  static constexpr bool stochastic = true;
  __device__ __host__ static float to_float(fp16s_t v) { return (float)v.v; }
  __device__ __host__ static fp16s_t from_float(float v) { return fp16s_t{(_Float16)v}; }
  // gfx950's stochastic-rounding conversion (v_cvt_sr_f16_f32): the top bits
  // of r, as many as the FP32 pattern carries below the FP16 spacing of |f|,
  // are added to those bits before truncation, so the value rounds up with
  // probability equal to its distance from the lower neighbour (checked on
  // the device: always a neighbour, unbiased, decided by the high bits).
  __device__ static fp16s_t from_float_sr(float f, uint32_t r) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 v = __builtin_amdgcn_cvt_sr_f16_f32(h2{0, 0}, f, r, false);
    return fp16s_t{v[0]};
  }
};
template <>
struct Storage<bf16s_t> {
  using compute = float;
  static constexpr bool scaled = true;
  static constexpr bool stochastic = true;
  __device__ __host__ static float to_float(bf16s_t v) {
    return __builtin_bit_cast(float, (uint32_t)v.u << 16);
  }
  __device__ __host__ static bf16s_t from_float(float f) {
    return bf16s_t{Storage<bf16_t>::from_float(f).u};
  }
  // BF16 is the top half of FP32: gfx950's v_cvt_sr_bf16_f32 adds the top
  // 16 bits of r to the low half of the pattern and truncates, which rounds
  // the magnitude stochastically.
  __device__ static bf16s_t from_float_sr(float f, uint32_t r) {
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    const b2 v = __builtin_amdgcn_cvt_sr_bf16_f32(b2{0, 0}, f, r, false);
    return bf16s_t{__builtin_bit_cast(uint16_t, v[0])};
  }
};

template <typename S>
struct IsStochastic {
  static constexpr bool value = false;
};
template <>
struct IsStochastic<fp16s_t> {
  static constexpr bool value = true;
};
template <>
struct IsStochastic<bf16s_t> {
  static constexpr bool value = true;
};

// Counter-based random word for (cell, direction, step seed): C. Wellons'
// published "lowbias32" 32-bit integer hash (two xor-shift / multiply
// rounds, public domain).
__device__ __host__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

template <typename S>
struct ComputeOf {
  using type = typename Storage<S>::compute;
};

// Factor that turns a stored value of direction k into g_k (1 unless scaled).
template <typename S, int K>
__device__ __forceinline__ typename ComputeOf<S>::type decode_factor(double inv_sigma) {
  using C = typename ComputeOf<S>::type;
  if constexpr (Storage<S>::scaled) return (C)(kLat.w[K] * inv_sigma);
  else return (C)1;
}
template <typename S, int K>
__device__ __forceinline__ typename ComputeOf<S>::type encode_factor(double sigma) {
  using C = typename ComputeOf<S>::type;
  if constexpr (Storage<S>::scaled) return (C)(sigma / kLat.w[K]);
  else return (C)1;
}
// Runtime-k versions for the set-up kernels.
__device__ __host__ inline double weight_of(int k) { return k == 0 ? 1.0 / 3.0 : (k < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

// ---------------------------------------------------------------- collision
// Input: post-streaming deviations g[19]; output overwrites g.

template <typename C>
__device__ __forceinline__ void moments(const C* g, C& rho, C& ux, C& uy, C& uz) {
  rho = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) +
        ((g[8] + g[9]) + (g[10] + g[11])) + ((g[12] + g[13]) + (g[14] + g[15])) +
        ((g[16] + g[17]) + g[18]);
  ux = ((g[1] - g[2]) + (g[7] - g[10])) + ((g[9] - g[8]) + (g[11] - g[14])) + (g[13] - g[12]);
  uy = ((g[3] - g[4]) + (g[7] - g[10])) + ((g[8] - g[9]) + (g[15] - g[18])) + (g[17] - g[16]);
  uz = ((g[5] - g[6]) + (g[11] - g[14])) + ((g[12] - g[13]) + (g[15] - g[18])) + (g[16] - g[17]);
}

// Deviation equilibrium w_k {drho + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u}.
template <typename C, int K>
__device__ __forceinline__ C geq(C rho, C ux, C uy, C uz, C usq) {
  constexpr C w = (C)kLat.w[K];
  const C eu = (C)kLat.ex[K] * ux + (C)kLat.ey[K] * uy + (C)kLat.ez[K] * uz;
  return w * (rho + (C)3 * eu + (C)4.5 * eu * eu - (C)1.5 * usq);
}

template <typename C>
__device__ __forceinline__ void collide_srt(C* g, C omega) {
  C rho, ux, uy, uz;
  moments(g, rho, ux, uy, uz);
  const C usq = ux * ux + uy * uy + uz * uz;
#define LBM_SRT(K) g[K] = g[K] - omega * (g[K] - geq<C, K>(rho, ux, uy, uz, usq));
  LBM_SRT(0) LBM_SRT(1) LBM_SRT(2) LBM_SRT(3) LBM_SRT(4) LBM_SRT(5) LBM_SRT(6) LBM_SRT(7)
  LBM_SRT(8) LBM_SRT(9) LBM_SRT(10) LBM_SRT(11) LBM_SRT(12) LBM_SRT(13) LBM_SRT(14)
  LBM_SRT(15) LBM_SRT(16) LBM_SRT(17) LBM_SRT(18)
#undef LBM_SRT
}

// TRT (eq. (TRT)): symmetric part relaxed with omega+, antisymmetric with
// omega-, per opposite pair (k, kb).
template <typename C, int K, int KB>
__device__ __forceinline__ void trt_pair(C* g, C rho, C ux, C uy, C uz, C usq, C wp, C wm) {
  constexpr C w = (C)kLat.w[K];
  const C eu = (C)kLat.ex[K] * ux + (C)kLat.ey[K] * uy + (C)kLat.ez[K] * uz;
  const C eq_p = w * (rho + (C)4.5 * eu * eu - (C)1.5 * usq);
  const C eq_m = w * (C)3 * eu;
  const C dp = wp * ((C)0.5 * (g[K] + g[KB]) - eq_p);
  const C dm = wm * ((C)0.5 * (g[K] - g[KB]) - eq_m);
  g[K] = g[K] - dp - dm;
  g[KB] = g[KB] - dp + dm;
}

template <typename C>
__device__ __forceinline__ void collide_trt(C* g, C wp, C wm) {
  C rho, ux, uy, uz;
  moments(g, rho, ux, uy, uz);
  const C usq = ux * ux + uy * uy + uz * uz;
  g[0] = g[0] - wp * (g[0] - (C)kLat.w[0] * (rho - (C)1.5 * usq));
  trt_pair<C, 1, 2>(g, rho, ux, uy, uz, usq, wp, wm);
  trt_pair<C, 3, 4>(g, rho, ux, uy, uz, usq, wp, wm);
  trt_pair<C, 5, 6>(g, rho, ux, uy, uz, usq, wp, wm);
  trt_pair<C, 7, 10>(g, rho, ux, uy, uz, usq, wp, wm);
  trt_pair<C, 8, 9>(g, rho, ux, uy, uz, usq, wp, wm);
  trt_pair<C, 11, 14>(g, rho, ux, uy, uz, usq, wp, wm);
  trt_pair<C, 12, 13>(g, rho, ux, uy, uz, usq, wp, wm);
  trt_pair<C, 15, 18>(g, rho, ux, uy, uz, usq, wp, wm);
  trt_pair<C, 16, 17>(g, rho, ux, uy, uz, usq, wp, wm);
}

// MRT (eq. (MRT)) as g* = g - M^-1 S M (g - g^eq) with M^-1 = M^T diag(1/|M_i|^2).
// M is a compile-time constant; the unrolled products fold its zeros.
// Conserved moments (rows 0, 3, 5, 7) carry no non-equilibrium part.
// Rows of M that are even under e -> -e (the rest are odd).  The moving
// directions form 9 opposite pairs (kPairA[p], opp), so an even row sees only
// the pair sums and an odd row only the pair differences, and the
// back-transform of a pair is one even and one odd sum: about half the
// multiply-adds of the dense product.
constexpr bool mrt_even_row(int i) { return i <= 2 || (i >= 9 && i <= 15); }
constexpr int kPairA[9] = {1, 3, 5, 7, 8, 11, 12, 15, 16};

constexpr bool mrt_pair_structure_holds() {
  bool seen[kQ] = {};
  for (int p = 0; p < 9; ++p) {
    const int a = kPairA[p], b = kLat.opp[a];
    if (a == b || seen[a] || seen[b]) return false;
    seen[a] = seen[b] = true;
  }
  for (int i = 0; i < kQ; ++i) {
    if (!mrt_even_row(i) && kMrt.m[i][0] != 0.0) return false;
    for (int k = 1; k < kQ; ++k) {
      const double sgn = mrt_even_row(i) ? 1.0 : -1.0;
      if (kMrt.m[i][k] != sgn * kMrt.m[i][kLat.opp[k]]) return false;
    }
  }
  return true;
}
static_assert(mrt_pair_structure_holds(), "MRT rows must be even or odd over opposite pairs");

template <typename C>
__device__ __forceinline__ void collide_mrt(C* g, C s_nu, C s_e, C s_zeta) {
  C rho, ux, uy, uz;
  moments(g, rho, ux, uy, uz);
  const C usq = ux * ux + uy * uy + uz * uz;
  C d[kQ];
  d[0] = g[0] - geq<C, 0>(rho, ux, uy, uz, usq);
#define LBM_D(K) d[K] = g[K] - geq<C, K>(rho, ux, uy, uz, usq);
  LBM_D(1) LBM_D(2) LBM_D(3) LBM_D(4) LBM_D(5) LBM_D(6) LBM_D(7) LBM_D(8) LBM_D(9)
  LBM_D(10) LBM_D(11) LBM_D(12) LBM_D(13) LBM_D(14) LBM_D(15) LBM_D(16) LBM_D(17) LBM_D(18)
#undef LBM_D
  // pair sums and differences of the non-equilibrium part
  C ps[9], pd[9];
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    ps[p] = d[kPairA[p]] + d[kLat.opp[kPairA[p]]];
    pd[p] = d[kPairA[p]] - d[kLat.opp[kPairA[p]]];
  }
  // relaxed moments r_i = s_i (M d)_i / |M_i|^2 (conserved moments: 0)
  C r[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    if (i == 0 || i == 3 || i == 5 || i == 7) {
      r[i] = (C)0;
      continue;
    }
    C m = (C)0;
    if (mrt_even_row(i)) {
      if (kMrt.m[i][0] != 0.0) m += (C)kMrt.m[i][0] * d[0];
#pragma unroll
      for (int p = 0; p < 9; ++p)
        if (kMrt.m[i][kPairA[p]] != 0.0) m += (C)kMrt.m[i][kPairA[p]] * ps[p];
    } else {
#pragma unroll
      for (int p = 0; p < 9; ++p)
        if (kMrt.m[i][kPairA[p]] != 0.0) m += (C)kMrt.m[i][kPairA[p]] * pd[p];
    }
    const C s = (i == 1 || i == 2) ? s_e
                : (i == 9 || i == 11 || i == 13 || i == 14 || i == 15) ? s_nu
                                                                     : s_zeta;
    r[i] = s * m * (C)(1.0 / kMrt.n2[i]);
  }
  // g_k -= sum_i M_ik r_i, as an even and an odd part per pair
  {
    C a = (C)0;
#pragma unroll
    for (int i = 1; i < kQ; ++i)
      if (mrt_even_row(i) && kMrt.m[i][0] != 0.0) a += (C)kMrt.m[i][0] * r[i];
    g[0] = g[0] - a;
  }
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    const int ka = kPairA[p], kb = kLat.opp[ka];
    C ae = (C)0, ao = (C)0;
#pragma unroll
    for (int i = 1; i < kQ; ++i) {
      if (i == 3 || i == 5 || i == 7 || kMrt.m[i][ka] == 0.0) continue;
      if (mrt_even_row(i))
        ae += (C)kMrt.m[i][ka] * r[i];
      else
        ao += (C)kMrt.m[i][ka] * r[i];
    }
    g[ka] = g[ka] - (ae + ao);
    g[kb] = g[kb] - (ae - ao);
  }
}

// Set-up and reduction kernels convert one stored value at a runtime k.
template <typename S>
__device__ __forceinline__ double stored_to_g(S v, int k, double sigma) {
  const double f = (double)Storage<S>::to_float(v);
  return Storage<S>::scaled ? f * (weight_of(k) / sigma) : f;
}
template <typename S>
__device__ __forceinline__ S g_to_stored(double g, int k, double sigma) {
  using C = typename Storage<S>::compute;
  return Storage<S>::from_float((C)(Storage<S>::scaled ? g * (sigma / weight_of(k)) : g));
}

// ------------------------------------------------------------ reductions
// FP64 sums over fluid cells: [0..2] sum u, [3] sum drho, [4] max |u|^2,
// [5] count of non-finite cells.  Deterministic: fixed grid, fixed per-thread
// order, fixed trees, no atomics.

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;
constexpr int kRedVals = 8;
// Largest workgroups that call block_reduce: the single-domain step
// (kStepThreads, up to 16 wavefronts of one tile each) and the batch step
// (kBatchThreads, whose shape the autotuner searches up to this size).
// block_reduce keeps one LDS slot per wavefront.
constexpr int kStepThreads = 1024;
constexpr int kBatchThreads = 1024;
constexpr int kMaxWaves = kBatchThreads / 64;
static_assert(kMaxWaves * 64 >= kStepThreads && kMaxWaves * 64 >= kBatchThreads &&
                  kMaxWaves * 64 >= kRedThreads,
              "block_reduce needs an LDS slot for every wavefront of the largest block");

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}

// Block reduction of NV doubles (kind 0 = sum, 1 = max): wavefront shuffles,
// then one LDS slot per wavefront folded in wavefront order.  Every thread of
// the block must call it.
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], const int (&kind)[NV], double* out) {
  __shared__ double sh[kMaxWaves][NV];
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int nwaves = (blockDim.x * blockDim.y + 63) >> 6;
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = kind[i] ? wave_max(v[i]) : wave_sum(v[i]);
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[wv][i] = v[i];
  __syncthreads();
  if (tid < NV) {
    const int i = tid;
    double a = sh[0][i];
    for (int w = 1; w < nwaves; ++w) a = kind[i] ? fmax(a, sh[w][i]) : a + sh[w][i];
    out[i] = a;
  }
}

// ---------------------------------------------------------------- the step

// Address of the node at (x + dx, y + dy, z + dz) given the tiled-address
// parts of the thread's wrapped neighbour coordinates.
struct Nbr {
  int xs[3];  // x parts of x - 1, x, x + 1 (wrapped)
  int ys[3];  // y parts of y - 1, y, y + 1 (wrapped)
  int zs[3];  // plane offsets of z - 1, z, z + 1 (wrapped)
  __device__ __forceinline__ int at(int dx, int dy, int dz) const {
    return xs[dx + 1] + ys[dy + 1] + zs[dz + 1];
  }
};

// Weight class of direction k: 0 rest, 1 axis, 2 diagonal.
__device__ __host__ constexpr int wclass(int k) { return k == 0 ? 0 : (k < 7 ? 1 : 2); }

// Cell m steps from (x, y, z) along e_k, wrapped into the box; cross = +1
// when the unwrapped x is >= nx, -1 when < 0 (the read crosses the
// x-periodic plane and carries the density jump).
struct FarNode {
  int c;
  int cross;
};
__device__ __forceinline__ int wrap_into(int i, int n) { return ((i % n) + n) % n; }
__device__ __forceinline__ FarNode far_node(const StepParams& p, int x, int y, int z, int k,
                                            int m) {
  const int X = x + m * kLat.ex[k];
  FarNode f;
  f.cross = X >= p.nx ? 1 : (X < 0 ? -1 : 0);
  f.c = p.t.at(wrap_into(X, p.nx), wrap_into(y + m * kLat.ey[k], p.ny),
               wrap_into(z + m * kLat.ez[k], p.nz));
  return f;
}

// Population kk at a far node, with the jump of a crossing read.
template <typename S, typename C>
__device__ __forceinline__ C far_value(const S* __restrict__ src, const StepParams& p, FarNode f,
                                       int kk) {
  C v = (C)Storage<S>::to_float(src[state_slot<S>(p.t, kk, f.c)]);
  const C jw = (C)(wclass(kk) == 1 ? p.jump_axis : p.jump_diag);
  if (f.cross > 0) v -= jw;
  if (f.cross < 0) v += jw;
  return v;
}

// Density deviation and velocity of the stored (post-collision) state at
// cell c; collision conserves both, so these are the moments at time t_n.
template <typename S, typename C>
__device__ __forceinline__ void stored_moments(const S* __restrict__ src, const Tiling& t, int c,
                                               C& drho, C (&u)[3]) {
  drho = (C)0;
  u[0] = u[1] = u[2] = (C)0;
#pragma unroll
  for (int kk = 0; kk < kQ; ++kk) {
    const C v = (C)Storage<S>::to_float(src[state_slot<S>(t, kk, c)]);
    drho += v;
    u[0] += (C)kLat.ex[kk] * v;
    u[1] += (C)kLat.ey[kk] * v;
    u[2] += (C)kLat.ez[kk] * v;
  }
}

// Incoming value of direction k at fluid node (x, y, z), cell c, whose pull
// source is solid, for the interpolated rules of Sec. 2.2.1 (eqs. (LIBB),
// (QIBB), (fstar)-(IEBB), (MR), (CLI)) in the pull form: j = opp(k) points
// into the wall, x_f2 = x + e_k and x_f3 = x + 2 e_k lie away from it, and
// every right-hand side is a post-collision value of the stored state.  MR
// uses kappa_1 = (1 - 2q - 2q^2)/(1 + q)^2 (exact for linear profiles).  A
// rule that needs a solid node falls back: x_f2 solid -> bounce-back (LIBB
// and QIBB with q >= 1/2 keep LIBB's q >= 1/2 branch, which needs x_f1
// only); x_f3 solid -> LIBB (from QIBB) or CLI (from MR).  Unscaled storage
// (FP32, FP64) only.  m1 holds the density deviation and velocity of the
// stored state at x (IEBB only), own_j and own_k the stored g_j and g_k at x
// (the caller loads them once per node).
template <typename S, typename C>
__device__ C general_wall_value(const S* __restrict__ src, const uint32_t* __restrict__ flags,
                                const StepParams& p, int x, int y, int z, int c, int k, C q,
                                uint32_t fl, const C (&m1)[4], C pulled_j, C own_j, C own_k) {
  const int j = kLat.opp[k];
  const FarNode n2 = far_node(p, x, y, z, k, 1);
  const FarNode n3 = far_node(p, x, y, z, k, 2);
  // x_f2 = x - e_j is the pull source of direction j here, and x_f3 that of
  // direction j at x_f2, so the flag bits j of x and of x_f2 tell if they
  // are solid
  const bool f2 = !(fl & (1u << j));
  int rule = p.wall;
  // x_f3's flag word is read only by the rules that use x_f3
  const bool wants_f3 = rule == kRuleMR || (rule == kRuleQIBB && q < (C)0.5);
  const bool f3 = f2 && wants_f3 && !(flags[n2.c] & (1u << j));
  // g_j at x_f2 is this node's pull in direction j (pulled_j, raw); with the
  // jump of a read across the x-periodic plane
  C f2_j = pulled_j;
  {
    const C jw = (C)(wclass(j) == 1 ? p.jump_axis : p.jump_diag);
    if (n2.cross > 0) f2_j -= jw;
    if (n2.cross < 0) f2_j += jw;
  }
  if (rule == kRuleMR && !f3) rule = kRuleCLI;
  if (rule == kRuleQIBB && (q < (C)0.5 ? !f3 : !f2)) rule = kRuleLIBB;
  const C one = (C)1, two = (C)2;
  switch (rule) {
    case kRuleCLI: {
      if (!f2) return own_j;
      const C a = (one - two * q) / (one + two * q);
      return a * f2_j - a * own_k + own_j;
    }
    case kRuleLIBB:
      if (q < (C)0.5) {
        if (!f2) return own_j;
        return (one - two * q) * f2_j + two * q * own_j;
      }
      return (one - one / (two * q)) * own_k + own_j / (two * q);
    case kRuleQIBB:
      if (q < (C)0.5)
        return q * (one + two * q) * own_j +
               (one - (C)4 * q * q) * f2_j -
               q * (one - two * q) * far_value<S, C>(src, p, n3, j);
      return (two * q - one) / q * own_k + own_j / (q * (two * q + one)) +
             (one - two * q) / (two * q + one) * far_value<S, C>(src, p, n2, k);
    case kRuleIEBB: {
      const C drho1 = m1[0], u1[3] = {m1[1], m1[2], m1[3]};
      C ubf[3], X;
      const C tau = (C)(1.0 / p.omega_p);
      if (q < (C)0.5) {
        if (!f2) return own_j;
        if (p.side_in) {
          // written for x_f2 by the step that produced the source state
          const C* u2 = static_cast<const C*>(p.side_in) + 4LL * n2.c;
          ubf[0] = u2[0];
          ubf[1] = u2[1];
          ubf[2] = u2[2];
        } else {
          C d2;
          stored_moments<S, C>(src, p.t, n2.c, d2, ubf);
        }
        X = (two * q - one) / (tau - two);
      } else {
        const C f = one - (C)3 / (two * q);
        ubf[0] = f * u1[0];
        ubf[1] = f * u1[1];
        ubf[2] = f * u1[2];
        X = (two * q - one) / (tau + (C)0.5);
      }
      const C eub = (C)kLat.ex[j] * ubf[0] + (C)kLat.ey[j] * ubf[1] + (C)kLat.ez[j] * ubf[2];
      const C eu1 = (C)kLat.ex[j] * u1[0] + (C)kLat.ey[j] * u1[1] + (C)kLat.ez[j] * u1[2];
      const C uu = u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2];
      const C fstar =
          (C)kLat.w[j] * (drho1 + (C)3 * eub + (C)4.5 * eu1 * eu1 - (C)1.5 * uu);
      return (one - X) * own_j + X * fstar;
    }
    case kRuleMR: {
      if (!f2) return own_j;
      const C d = (one + q) * (one + q);
      const C k1 = (one - two * q - two * q * q) / d, k2 = q * q / d;
      return k1 * f2_j + k2 * far_value<S, C>(src, p, n3, j) -
             k1 * own_k - k2 * far_value<S, C>(src, p, n2, k) + own_j;
    }
    default:
      return own_j;
  }
}


// A parameter in the compute precision: FP64 kernels use the double, the
// others the FP32 copy that the host rounded.
template <typename C>
__device__ __forceinline__ C prm(double d, float f) {
  if constexpr (sizeof(C) == sizeof(float))
    return f;
  else
    return d;
}

// Pressure jump of direction k in the units of the stored values (g units
// for FP32 and FP64, g * sigma / w_k for the 16-bit formats).
template <typename S>
__device__ __forceinline__ typename ComputeOf<S>::type jump_stored(const StepParams& p, int k) {
  using C = typename ComputeOf<S>::type;
  const C j = wclass(k) == 1 ? prm<C>(p.jump_axis, p.jump_axisf) : prm<C>(p.jump_diag, p.jump_diagf);
  if constexpr (Storage<S>::scaled)
    return j * (C)p.enc[wclass(k)];
  else
    return j;
}

// The part of a node's time step after the pull: SBB / CLI wall links (the
// general rules are applied by the caller), pressure jump and collision.  g
// holds the pulled raw stored values (on a wall link: the stored coefficient
// a for CLI); own holds the node's own stored values of directions 1..18
// when it has wall links.  edge_x must be true when a lane of the wavefront
// lies on the box's x faces (x = 0 or nx - 1); it is wavefront-uniform, so
// the wavefronts inside the box skip the jump's per-lane tests.  On return g
// holds the new values in stored units, not yet rounded to the storage type;
// mom the pre-collision moments (which the collision conserves) and
// max_k |g*_k| / w_k of the result, for the optional reduction.
template <typename S, int COLL, int WALL>
__device__ __forceinline__ void finish_values(typename ComputeOf<S>::type (&g)[kQ],
                                              const S (&own)[kQ], const StepParams& p, int x,
                                              uint32_t fl, bool edge_x,
                                              typename ComputeOf<S>::type (&mom)[5]) {
  using C = typename ComputeOf<S>::type;
  using St = Storage<S>;
  static_assert(!(St::scaled && WALL == kGEN), "16-bit storage: SBB and CLI walls only");
  const int nx = p.nx;
  if constexpr (WALL != kGEN) {
    if (fl & kLinkMask) {
      // in stored units: every term of a link's value is a value of
      // direction k or of its opposite j, which share a weight and so a
      // storage scale
#pragma unroll
      for (int k = 1; k < kQ; ++k) {
        if (fl & (1u << k)) {
          const int j = kLat.opp[k];
          const C own_j = (C)St::to_float(own[j]);
          if constexpr (WALL == kCLI) {
            const C a = g[k];
            const C own_k = (C)St::to_float(own[k]);
            // g_j at the second node x_f2 = x + e_k (away from the wall) is
            // what this node pulls in direction j, so g[j] already holds it
            // (raw); it is read across the x-periodic plane with the pressure
            // jump.  If x_f2 is solid, g[j] is a coefficient and a = 0.
            C far_j = g[j];
            if (kLat.ex[k] == 1 && x == nx - 1) far_j -= jump_stored<S>(p, k);
            if (kLat.ex[k] == -1 && x == 0) far_j += jump_stored<S>(p, k);
            g[k] = a * far_j - a * own_k + own_j;
          } else {
            g[k] = own_j;
          }
        }
      }
    }
  }
  if constexpr (St::scaled) {
#pragma unroll
    for (int k = 0; k < kQ; ++k) g[k] *= (C)p.dec[wclass(k)];
  }

  // periodic pressure drop on pulls across the x-plane (not on wall links)
  if (edge_x) {
    if (x == 0) {
      const C ja = prm<C>(p.jump_axis, p.jump_axisf), jd = prm<C>(p.jump_diag, p.jump_diagf);
      if (!(fl & (1u << 1))) g[1] += ja;
      if (!(fl & (1u << 7))) g[7] += jd;
      if (!(fl & (1u << 9))) g[9] += jd;
      if (!(fl & (1u << 11))) g[11] += jd;
      if (!(fl & (1u << 13))) g[13] += jd;
    }
    if (x == nx - 1) {
      const C ja = prm<C>(p.jump_axis, p.jump_axisf), jd = prm<C>(p.jump_diag, p.jump_diagf);
      if (!(fl & (1u << 2))) g[2] -= ja;
      if (!(fl & (1u << 8))) g[8] -= jd;
      if (!(fl & (1u << 10))) g[10] -= jd;
      if (!(fl & (1u << 12))) g[12] -= jd;
      if (!(fl & (1u << 14))) g[14] -= jd;
    }
  }

  moments(g, mom[0], mom[1], mom[2], mom[3]);
  if constexpr (COLL == kSRT) {
    collide_srt<C>(g, prm<C>(p.omega_p, p.omega_pf));
  } else if constexpr (COLL == kTRT) {
    collide_trt<C>(g, prm<C>(p.omega_p, p.omega_pf), prm<C>(p.omega_m, p.omega_mf));
  } else {
    collide_mrt<C>(g, prm<C>(p.omega_p, p.omega_pf), prm<C>(p.s_e, p.s_ef),
                   prm<C>(p.s_zeta, p.s_zetaf));
  }
  C m = (C)0;
#pragma unroll
  for (int k = 0; k < kQ; ++k) m = fmax(m, fabs(g[k]) * (C)(1.0 / kLat.w[k]));
  mom[4] = m;
  if constexpr (St::scaled) {
#pragma unroll
    for (int k = 0; k < kQ; ++k) g[k] *= (C)p.enc[wclass(k)];
  }
}

// Stochastic rounding's random words: one finalised hash per cell and step,
// then direction k takes the high bits of (base + k * golden) * odd constant
// (multiplicative hashing).
__device__ __forceinline__ uint32_t sr_base(int c, unsigned seed) {
  return hash32((uint32_t)c * 19u + seed);
}
__device__ __forceinline__ uint32_t sr_word(uint32_t base, int k) {
  return (base + (uint32_t)k * 0x9e3779b9u) * 0x85ebca6bu;
}

// Round a node's new values (stored units) to the storage type.
template <typename S>
__device__ __forceinline__ void round_node(const typename ComputeOf<S>::type (&v)[kQ],
                                           const StepParams& p, int c, S (&out)[kQ]) {
  using St = Storage<S>;
  if constexpr (IsStochastic<S>::value) {
    const uint32_t base = sr_base(c, p.seed);
#pragma unroll
    for (int k = 0; k < kQ; ++k) out[k] = St::from_float_sr(v[k], sr_word(base, k));
  } else {
#pragma unroll
    for (int k = 0; k < kQ; ++k) out[k] = St::from_float(v[k]);
  }
}

template <typename S, int COLL, int WALL>
__device__ __forceinline__ void finish_node(typename ComputeOf<S>::type (&g)[kQ],
                                            const S (&own)[kQ], S (&out)[kQ],
                                            const StepParams& p, int x, int c, uint32_t fl,
                                            bool edge_x,
                                            typename ComputeOf<S>::type (&mom)[5]) {
  finish_values<S, COLL, WALL>(g, own, p, x, fl, edge_x, mom);
  round_node<S>(g, p, c, out);
}

// One time step for the node (x, y, z), fluid, with flag word fl: pull (one
// lane, one node), the general wall rules, then finish_node (edge_x as
// there).  SPLIT selects pulls from scalar per-direction bases plus 32-bit
// lane offsets (state_at); without it every lane forms 64-bit addresses.
// The split form needs about 40 more scalar registers; in the kernels with
// the general wall rules it made the compiler spill scalar registers (5-11%
// slower at 512^3), and the batch kernel, whose cell base comes from a table,
// got no scalar-base loads from it and was 1% slower, so only the
// single-domain SBB / CLI kernels use it.
template <typename S, int COLL, int WALL, bool SPLIT>
__device__ __forceinline__ void update_node(const S* __restrict__ src, S (&out)[kQ],
                                            const uint32_t* __restrict__ flags,
                                            const StepParams& p, int x, int y, int z, int c,
                                            uint32_t fl, bool edge_x,
                                            typename ComputeOf<S>::type (&mom)[5]) {
  using C = typename ComputeOf<S>::type;
  using St = Storage<S>;
  const int nx = p.nx, plane = p.t.plane;
  Nbr n;
  n.xs[0] = p.t.xpart(x == 0 ? nx - 1 : x - 1);
  n.xs[1] = p.t.xpart(x);
  n.xs[2] = p.t.xpart(x == nx - 1 ? 0 : x + 1);
  n.ys[0] = p.t.ypart(y == 0 ? p.ny - 1 : y - 1);
  n.ys[1] = p.t.ypart(y);
  n.ys[2] = p.t.ypart(y == p.ny - 1 ? 0 : y + 1);
  n.zs[0] = (z == 0 ? p.nz - 1 : z - 1) * plane;
  n.zs[1] = z * plane;
  n.zs[2] = (z == p.nz - 1 ? 0 : z + 1) * plane;

  C g[kQ];
  // pull: direction k arrives from x - e_k (raw stored values)
#pragma unroll
  for (int k = 0; k < kQ; ++k) {
    if constexpr (SPLIT)
      g[k] = (C)St::to_float(*state_at<S>(src, p.t, k, n.zs[1 - kLat.ez[k]],
                                          n.xs[1 - kLat.ex[k]] + n.ys[1 - kLat.ey[k]]));
    else
      g[k] = (C)St::to_float(
          *state_ptr<S>(src, p.t, k, n.at(-kLat.ex[k], -kLat.ey[k], -kLat.ez[k])));
  }

  // wall links: the pulled raw value is the stored coefficient a (CLI) or
  // the wall distance q (general rules)
  S own[kQ];
  if (fl & kLinkMask) {
    // The node's own stored values of every moving direction (the wall rules
    // need g_j and g_k at x), all requested before the first use: one memory
    // round trip per boundary node instead of one per link direction (512^3
    // sphere pack, FP32 CLI: 2.84 -> 2.56 ms per step).  IEBB's moments at x
    // come from the same values.  (64-bit lane addresses: with scalar bases
    // per direction as for the pulls, the boundary wavefronts' extra scalar
    // work made the 512^3 sphere-pack step 3% slower.)
#pragma unroll
    for (int k = 1; k < kQ; ++k) own[k] = *state_ptr<S>(src, p.t, k, c);
    if constexpr (WALL == kGEN) {
      C m1[4] = {(C)0, (C)0, (C)0, (C)0};
      if (p.wall == kRuleIEBB) {
        own[0] = src[state_slot<S>(p.t, 0, c)];
#pragma unroll
        for (int kk = 0; kk < kQ; ++kk) {
          const C v = (C)St::to_float(own[kk]);
          m1[0] += v;
          m1[1] += (C)kLat.ex[kk] * v;
          m1[2] += (C)kLat.ey[kk] * v;
          m1[3] += (C)kLat.ez[kk] * v;
        }
      }
      // the pulled raw value is the link's wall distance q.  g[j] may already
      // hold a wall value when direction j is a link too; the rules use the
      // pull g[j] only when x_f2 = x - e_j is fluid, i.e. j is no link.
#pragma unroll
      for (int k = 1; k < kQ; ++k) {
        if (fl & (1u << k)) {
          const int j = kLat.opp[k];
          g[k] = general_wall_value<S, C>(src, flags, p, x, y, z, c, k, g[k], fl, m1, g[j],
                                          (C)St::to_float(own[j]), (C)St::to_float(own[k]));
        }
      }
    }
  }
  finish_node<S, COLL, WALL>(g, own, out, p, x, c, fl, edge_x, mom);
}

// The 19 values a solid cell writes: its wall-link slots (flag bit k: the
// slot in plane k is pulled by the fluid node c + e_k and holds that link's
// coefficient) are copied, every other slot is zero.  In batches, solid
// cells that share a tile or a line with fluid cells may write so that the
// lines the fluid cells write are written whole: where sphere surfaces cut
// many lines,
// partly written lines cost far more than their bytes (a batch of 64^3 cells
// holding spheres of diameter 50 steps 17% faster with mode 1).
template <typename S>
__device__ __forceinline__ void solid_node(const S* __restrict__ src, S (&out)[kQ],
                                           const Tiling& t, int c, uint32_t fl) {
  out[0] = Storage<S>::from_float(0);
#pragma unroll
  for (int k = 1; k < kQ; ++k)
    out[k] = (fl & (1u << k)) ? src[state_slot<S>(t, k, c)] : Storage<S>::from_float(0);
}

// Whether this lane stores, given the fluid lanes of its wavefront: fluid
// lanes always; solid lanes never (mode 0), when the wavefront holds a fluid
// cell (mode 1), or when their 128-byte line of a plane does (mode 2: the
// lanes of a wavefront hold 64 consecutive addresses, so lanes [g, g + L)
// share a line, L = 128 / sizeof(S)).
template <typename S>
__device__ __forceinline__ bool solid_stores(int mode, bool solid, unsigned long long fluid) {
  if (!solid) return true;
  if (mode == 0) return false;
  if (mode == 1) return fluid != 0;
  constexpr int L = 128 / (int)sizeof(S);
  if constexpr (L >= 64) {
    return fluid != 0;
  } else {
    const int g = ((int)__lane_id() / L) * L;
    return ((fluid >> g) & ((1ull << L) - 1)) != 0;
  }
}

// Store a node's 19 values; NT selects non-temporal stores (the new state is
// not read again within this step).
template <typename S>
__device__ __forceinline__ void nontemporal_store(S v, S* p) {
  if constexpr (sizeof(S) == 2)  // the 16-bit formats as their bit patterns
    __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, v), reinterpret_cast<uint16_t*>(p));
  else
    __builtin_nontemporal_store(v, p);
}

template <typename S, bool NT, bool SPLIT>
__device__ __forceinline__ void store_node(S* __restrict__ dst, const S (&out)[kQ],
                                           const Tiling& t, long long zstart, int r) {
#pragma unroll
  for (int k = 0; k < kQ; ++k) {
    S* q = SPLIT ? state_at<S>(dst, t, k, zstart, r) : state_ptr<S>(dst, t, k, (int)zstart + r);
    if constexpr (NT)
      nontemporal_store(out[k], q);
    else
      *q = out[k];
  }
}

// IEBB's side buffer: a near-wall cell's velocity (the pre-collision
// momentum, which the collision conserves, i.e. that of the state written).
template <typename C>
__device__ __forceinline__ void store_side(const StepParams& p, uint8_t cls, int c,
                                           const C (&mom)[5]) {
  if (p.side_out && (cls & kClsNearWall)) {
    C* u = static_cast<C*>(p.side_out) + 4LL * c;
    u[0] = mom[1];
    u[1] = mom[2];
    u[2] = mom[3];
  }
}

// Cell of this thread in plane z: wavefront threadIdx.y of the block takes
// tile blockIdx.x * blockDim.y + threadIdx.y of the plane (tiles in row-major
// order), lane threadIdx.x its cell in the tile, so the lanes of a wavefront
// hold 64 consecutive addresses (tiles of 64 cells: batches).  inside is
// false for padding cells and for tiles past the end of the plane (c must
// not be used then).
struct TileCell {
  int x, y, c;  // coordinates and address
  int r;        // address within the z plane
  bool inside;
};
__device__ __forceinline__ TileCell tile_cell(const Tiling& t, int z) {
  const int tile = blockIdx.x * blockDim.y + threadIdx.y;
  const int l = threadIdx.x;
  const int tx = tile % t.ntx, ty = tile / t.ntx;
  TileCell r;
  r.x = (tx << t.tw_log2) + (l & ((1 << t.tw_log2) - 1));
  r.y = (ty << t.th_log2) + (l >> t.tw_log2);
  r.inside = ty < t.nty && r.x < t.nx && r.y < t.ny;
  r.r = (tile << 6) + l;
  r.c = r.r + z * t.plane;
  return r;
}

// Unit column and tile row of this wavefront in a step workgroup (the bw x
// bh arrangement of StepParams; the grid is nbx workgroups along a band of
// bh tile rows times the bands times the z planes).  Units past the row end
// give u >= units per row.
__device__ __forceinline__ void step_unit(const StepParams& p, int& u, int& ty) {
  const int j = threadIdx.y;
  u = blockIdx.x * p.bw + j % p.bw;
  ty = blockIdx.y * p.bh + j / p.bw;
}

// Partial-sum slot of a step workgroup.
__device__ __forceinline__ long long step_block_id() {
  return blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
}

// tile_cell for the single-domain step: the wavefront's unit is 64
// consecutive addresses of its tile row (a tile of 64 cells, or half of one
// of 128).
__device__ __forceinline__ TileCell step_tile_cell(const StepParams& p, int z) {
  const Tiling& t = p.t;
  int u, ty;
  step_unit(p, u, ty);
  const int tl = t.tile_log2();
  const int q = (u << 6) + threadIdx.x;  // address within the tile row
  const int tx = q >> tl, o = q & ((1 << tl) - 1);
  TileCell r;
  r.x = (tx << t.tw_log2) + (o & ((1 << t.tw_log2) - 1));
  r.y = (ty << t.th_log2) + (o >> t.tw_log2);
  r.inside = tx < t.ntx && ty < t.nty && r.x < t.nx && r.y < t.ny;
  r.r = ty * (t.ntx << tl) + q;
  r.c = r.r + z * t.plane;
  return r;
}

// Flag word of a cell from its class byte: only cells with wall links (or
// link slots, for solid cells) read the word.
__device__ __forceinline__ uint32_t flag_word(uint8_t k, const uint32_t* __restrict__ flags, int c) {
  if (k & kClsLinks) return flags[c];
  return (k & kClsSolid) ? kSolid : 0u;
}

// The fused stream-and-collide step over the box.  A block of blockDim.y
// wavefronts covers that many consecutive tiles of one z plane; with 16 x 4
// tiles and 8 wavefronts it spans 128 x 4 cells, so most of the lines that
// the +-1 shifted pulls share with neighbouring tiles are read by the same
// workgroup.  With RED the block also writes FP64 partial sums of the state
// it produced (u, drho, max |u|^2, non-finite count) to partials[block].  NT
// selects non-temporal stores (the new state is not read again in the step).
template <typename S, int COLL, int WALL, bool RED, bool NT>
__global__ __launch_bounds__(kStepThreads) void step_kernel(const S* __restrict__ src,
                                                            S* __restrict__ dst,
                                                            const uint8_t* __restrict__ cls,
                                                            const uint32_t* __restrict__ flags,
                                                            const StepParams p,
                                                            double* __restrict__ partials) {
  using C = typename ComputeOf<S>::type;
  constexpr bool kSplit = WALL != kGEN;  // (update_node)
  const int z = blockIdx.z;
  const TileCell tc = step_tile_cell(p, z);
  const uint8_t k = tc.inside ? cls[tc.c] : kClsSolid;
  const bool edge_x = __ballot(tc.x == 0 || tc.x == p.nx - 1) != 0;
  if constexpr (!RED) {
    if (k & kClsSolid) return;
    const uint32_t fl = flag_word(k, flags, tc.c);
    S out[kQ];
    C mom[5];
    update_node<S, COLL, WALL, kSplit>(src, out, flags, p, tc.x, tc.y, z, tc.c, fl, edge_x, mom);
    store_node<S, NT, kSplit>(dst, out, p.t, (long long)z * p.t.plane, tc.r);
    if constexpr (WALL == kGEN) store_side<C>(p, k, tc.c, mom);
  } else {
    double v[kRedVals] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (!(k & kClsSolid)) {
      const uint32_t fl = flag_word(k, flags, tc.c);
      S out[kQ];
      C mom[5];
      update_node<S, COLL, WALL, kSplit>(src, out, flags, p, tc.x, tc.y, z, tc.c, fl, edge_x,
                                         mom);
      store_node<S, NT, kSplit>(dst, out, p.t, (long long)z * p.t.plane, tc.r);
      if constexpr (WALL == kGEN) store_side<C>(p, k, tc.c, mom);
      const double rho = mom[0], ux = mom[1], uy = mom[2], uz = mom[3];
      const double u2 = ux * ux + uy * uy + uz * uz;
      v[0] = ux;
      v[1] = uy;
      v[2] = uz;
      v[3] = rho;
      if (isfinite(u2) && isfinite(rho))
        v[4] = u2;
      else
        v[5] = 1.0;
      v[6] = isfinite((double)mom[4]) ? (double)mom[4] : 0.0;
    }
    const int kind[kRedVals] = {0, 0, 0, 0, 1, 0, 1, 0};
    block_reduce<kRedVals>(v, kind, partials + step_block_id() * kRedVals);
  }
}

// ------------------------------------------- two cells per lane (16-bit storage)
// With 2-byte values a wavefront load of one value per lane moves 128 bytes,
// and even at the full 8 wavefronts per SIMD too few bytes are in flight to
// keep HBM busy (all-fluid 512^3 box: 0.50 of 8 TB/s against 0.64 for FP32).
// Here each lane takes the two x-adjacent cells of one aligned 4-byte word:
// a wavefront covers 128 consecutive addresses (a 32 x 4 tile) and loads 256
// bytes per direction.  A pull with e_x = 0 reads the word at the cells' own
// x; with e_x = +1 cell A (even x) needs the high half of the word to its
// left, which is the next lower lane's word (a DPP row shift) except at the
// start of a tile row or of a 16-lane DPP row, where the lane reads that word
// itself; e_x = -1 mirrors this.  The box edge in x must fall on a tile edge
// (nx a multiple of the tile width), so the periodic wrap only happens at the
// reads at tile edges.  A lane whose pair holds one solid cell stores that
// cell's own (unchanged) values with the fluid one.  Every cell goes through
// finish_values with its own coordinates and is rounded with its own random
// word, so the stored results are the one-cell kernel's.

// In-plane address of a pair wavefront's cell A and its coordinates.  The
// wavefront's unit u is the 128 consecutive addresses [128u, 128u + 128) of
// its tile row: one 32 x 4 tile (the layout of 16-bit states beyond 1 GiB),
// or two x-adjacent tiles of 64 cells (lanes 0-31 and 32-63).
struct PairCell {
  int a;             // in-plane address of cell A (even); cell B is a + 1
  int x, y;          // cell A (cell B is x + 1)
  bool inside;       // false for tiles past the row or plane and padding rows
  bool edge_lo;      // the word left of the pair is not in lane - 1 of the DPP row
  bool edge_hi;      // the word right of the pair is not in lane + 1
};
__device__ __forceinline__ PairCell pair_cell(const StepParams& p) {
  const Tiling& t = p.t;
  int u, ty;
  step_unit(p, u, ty);
  const int l = threadIdx.x;
  const int tl = t.tile_log2();
  const int q = (u << 7) + 2 * l;  // address within the tile row
  const int tx = q >> tl, o = q & ((1 << tl) - 1);
  const int xin = o & ((1 << t.tw_log2) - 1);
  PairCell r;
  r.a = ty * (t.ntx << tl) + q;
  r.x = (tx << t.tw_log2) + xin;
  r.y = (ty << t.th_log2) + (o >> t.tw_log2);
  r.inside = tx < t.ntx && ty < t.nty && r.y < t.ny;
  r.edge_lo = xin == 0 || (l & 15) == 0;
  r.edge_hi = xin == (1 << t.tw_log2) - 2 || (l & 15) == 15;
  return r;
}

template <typename S>
__device__ __forceinline__ S half_of(uint32_t w, int h) {
  return __builtin_bit_cast(S, (uint16_t)(w >> (16 * h)));
}
template <typename S>
__device__ __forceinline__ uint32_t bits_of(S v) {
  return (uint32_t)__builtin_bit_cast(uint16_t, v);
}

// Half h of a pair word set to v rounded to the 16-bit type S, the other
// half kept from w.  The stochastic formats round with the conversion
// instruction itself (its high-half form keeps the low half) and the cell's
// own random word r, so each half equals round_node's result for its cell.
template <typename S, int H>
__device__ __forceinline__ uint32_t put_half(uint32_t w, float v, uint32_t r) {
  if constexpr (std::is_same<S, fp16s_t>::value) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(
        uint32_t, __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(h2, w), v, r, H != 0));
  } else if constexpr (std::is_same<S, bf16s_t>::value) {
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(
        uint32_t, __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(b2, w), v, r, H != 0));
  } else {
    const uint32_t b = bits_of<S>(Storage<S>::from_float(v));
    return H ? (w & 0xffffu) | (b << 16) : (w & 0xffff0000u) | b;
  }
}

template <typename S, int COLL, int WALL, bool RED, bool NT>
__global__ __launch_bounds__(kStepThreads) void step_pair_kernel(const S* __restrict__ src,
                                                                 S* __restrict__ dst,
                                                                 const uint8_t* __restrict__ cls,
                                                                 const uint32_t* __restrict__ flags,
                                                                 const StepParams p,
                                                                 double* __restrict__ partials) {
  static_assert(sizeof(S) == 2, "two cells per lane: 16-bit storage only");
  static_assert(WALL != kGEN, "two cells per lane: SBB and CLI only");
  using C = typename ComputeOf<S>::type;
  const Tiling& t = p.t;
  const int z = blockIdx.z;
  const PairCell pc = pair_cell(p);
  const long long zplane = (long long)z * t.plane;  // address of plane z's first cell
  const int c = pc.a + (int)zplane;                 // cell A
  const uint32_t cl2 =
      pc.inside ? (uint32_t)(*reinterpret_cast<const uint16_t*>(cls + zplane + (uint32_t)pc.a))
                : (uint32_t)(kClsSolid | (kClsSolid << 8));
  const bool solid_a = cl2 & kClsSolid, solid_b = (cl2 >> 8) & kClsSolid;
  const bool live = !(solid_a && solid_b);
  const unsigned long long ball = __ballot(live);
  double v[kRedVals] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (ball != 0) {
    // the lanes of a DPP row with a fluid cell read their words (neighbours
    // within the row need them, solid or not)
    const bool row_reads = pc.inside && ((ball >> (threadIdx.x & 48)) & 0xffffull) != 0;
    const int nx = p.nx;
    // Word addresses as a wavefront-uniform base (direction plane k, source
    // z plane) plus a 32-bit byte offset per lane, twice the in-plane cell
    // address of the pair's even cell: the x parts of x - 2, x, x + 2 and
    // the y parts of y - 1, y, y + 1 (wrapped) are added once per (x, y)
    // combination.  Lanes that need no word read the plane's first word;
    // lanes at no tile or DPP-row edge read their own word for the edge load.
    const uint32_t xo = row_reads ? 2u * (uint32_t)t.xpart(pc.x) : 0u;
    const uint32_t xlo =
        row_reads && pc.edge_lo ? 2u * (uint32_t)t.xpart(pc.x == 0 ? nx - 2 : pc.x - 2) : xo;
    const uint32_t xhi =
        row_reads && pc.edge_hi ? 2u * (uint32_t)t.xpart(pc.x + 2 == nx ? 0 : pc.x + 2) : xo;
    uint32_t yo[3];
    yo[0] = row_reads ? 2u * (uint32_t)t.ypart(pc.y == 0 ? p.ny - 1 : pc.y - 1) : 0u;
    yo[1] = row_reads ? 2u * (uint32_t)t.ypart(pc.y) : 0u;
    yo[2] = row_reads ? 2u * (uint32_t)t.ypart(pc.y == p.ny - 1 ? 0 : pc.y + 1) : 0u;
    const long long zb[3] = {2LL * (z == 0 ? p.nz - 1 : z - 1) * t.plane, 2LL * zplane,
                             2LL * (z == p.nz - 1 ? 0 : z + 1) * t.plane};
    const char* sb = reinterpret_cast<const char*>(src);

    // pull: one word per direction with cell A's pulled value in the low
    // half and cell B's in the high half (direction k from x - e_k)
    // Every lane issues every load (no branches, so that all of them are in
    // flight together).  All loads come before the first DPP shift, which
    // waits for its word.
    uint32_t raw[kQ], edge[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
      const int ex = kLat.ex[k];
      // 16-bit states are direction planes: plane k, source z plane
      const char* bk = sb + 2LL * state_slot<S>(t, k, 0) + zb[1 - kLat.ez[k]];
      const uint32_t yk = yo[1 - kLat.ey[k]];
      raw[k] = *reinterpret_cast<const uint32_t*>(bk + (xo + yk));
      if (ex == 1) edge[k] = *reinterpret_cast<const uint32_t*>(bk + (xlo + yk));
      if (ex == -1) edge[k] = *reinterpret_cast<const uint32_t*>(bk + (xhi + yk));
    }
    // Boundary pairs: both flag words and the pair's own words, requested
    // with the pulls (one memory round trip): wall rules of link cells, and
    // the unchanged half of a pair with one solid cell (whose fluid partner
    // then has an x link).
    const uint32_t ab = 2u * (uint32_t)pc.a;
    const bool links = live && (cl2 & (kClsLinks | (kClsLinks << 8))) != 0;
    uint2 flw = make_uint2(0u, 0u);
    uint32_t own_w[kQ];
    if (links) {
      flw = *reinterpret_cast<const uint2*>(flags + c);
#pragma unroll
      for (int k = 0; k < kQ; ++k)
        own_w[k] = *reinterpret_cast<const uint32_t*>(sb + 2LL * state_slot<S>(t, k, 0) +
                                                      zb[1] + ab);
    }
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
      const int ex = kLat.ex[k];
      const uint32_t w = raw[k];
      if (ex == 1) {
        // A <- high half of the word on the left, B <- low half of w
        const uint32_t prev =
            (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x111, 0xf, 0xf, true);  // row_shr:1
        raw[k] = ((pc.edge_lo ? edge[k] : prev) >> 16) | (w << 16);
      } else if (ex == -1) {
        // A <- high half of w, B <- low half of the word on the right
        const uint32_t next =
            (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x101, 0xf, 0xf, true);  // row_shl:1
        raw[k] = (w >> 16) | ((pc.edge_hi ? edge[k] : next) << 16);
      }
    }

    // a lane of the wavefront on the box's x faces (cell A at x = 0, cell B
    // at x = nx - 1): wavefront-uniform
    const bool edge_x = __ballot(pc.x == 0 || pc.x + 2 == nx) != 0;
    C ga[kQ], gb[kQ];  // cell A (h = 0), cell B (h = 1)
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
      ga[k] = (C)Storage<S>::to_float(half_of<S>(raw[k], 0));
      gb[k] = (C)Storage<S>::to_float(half_of<S>(raw[k], 1));
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const bool solid = h ? solid_b : solid_a;
      C(&g)[kQ] = h ? gb : ga;
      if (!solid) {
        const uint32_t clh = (cl2 >> (8 * h)) & 0xffu;  // class bytes: A low, B high
        const uint32_t fl = (clh & kClsLinks) ? (h ? flw.y : flw.x) : 0u;
        S own[kQ];
#pragma unroll
        for (int k = 1; k < kQ; ++k) own[k] = half_of<S>(own_w[k], h);
        C mom[5];
        finish_values<S, COLL, WALL>(g, own, p, pc.x + h, fl, edge_x, mom);
        if constexpr (RED) {
          const double rho = mom[0], ux = mom[1], uy = mom[2], uz = mom[3];
          const double u2 = ux * ux + uy * uy + uz * uz;
          v[0] += ux;
          v[1] += uy;
          v[2] += uz;
          v[3] += rho;
          if (isfinite(u2) && isfinite(rho))
            v[4] = fmax(v[4], u2);
          else
            v[5] += 1.0;
          v[6] = fmax(v[6], isfinite((double)mom[4]) ? (double)mom[4] : 0.0);
        }
      }
    }
    // round into the pair words, cell A's half first (into the register of
    // A's value: the word's other initial bits are never used); every lane
    // rounds both halves, and a solid cell beside a fluid one then gets its
    // (constant) stored values back
    const uint32_t base_a = IsStochastic<S>::value ? sr_base(c, p.seed) : 0u;
    const uint32_t base_b = IsStochastic<S>::value ? sr_base(c + 1, p.seed) : 0u;
    uint32_t outw[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k)
      outw[k] = put_half<S, 1>(
          put_half<S, 0>(__builtin_bit_cast(uint32_t, ga[k]), ga[k], sr_word(base_a, k)),
          gb[k], sr_word(base_b, k));
    const bool mixed = links && solid_a != solid_b;
    if (__ballot(mixed) != 0 && mixed) {
      const uint32_t keep = solid_a ? 0x0000ffffu : 0xffff0000u;
#pragma unroll
      for (int k = 0; k < kQ; ++k) outw[k] = (own_w[k] & keep) | (outw[k] & ~keep);
    }
    if (live) {
      char* db = reinterpret_cast<char*>(dst);
#pragma unroll
      for (int k = 0; k < kQ; ++k) {
        uint32_t* q = reinterpret_cast<uint32_t*>(db + 2LL * state_slot<S>(t, k, 0) + zb[1] + ab);
        if constexpr (NT)
          __builtin_nontemporal_store(outw[k], q);
        else
          *q = outw[k];
      }
    }
  }
  if constexpr (RED) {
    const int kind[kRedVals] = {0, 0, 0, 0, 1, 0, 1, 0};
    block_reduce<kRedVals>(v, kind, partials + step_block_id() * kRedVals);
  }
}

// ------------------------------------------------------------ batches of cells
// B independent periodic cells of nx x ny x nz are stacked along z (cell b
// occupies addresses [b*cell_size, (b+1)*cell_size) of every direction plane,
// cell_size = nz planes of the cell's tiling).  Each block covers blockDim.y
// consecutive tiles of zper consecutive z planes of one cell (zper divides
// nz), reads that cell's parameters from a device table and skips inactive
// (converged or stopped) cells.  The grid's z runs over cell slots times the
// cell's z blocks: slot j is cell j, or with a list (the running cells in
// order, *n_list of them, rewritten by every convergence check) cell
// list[j], so that a run whose cells have mostly stopped launches blocks for
// the running ones only; slots from *n_list on return at once.  The partial
// sums of cell b form one segment of blocks_per_cell entries wherever its
// blocks ran.  p.solid_writes selects which solid cells also store
// (solid_stores, solid_node).

template <typename S, int COLL, int WALL, bool RED, bool NT>
__global__ __launch_bounds__(kBatchThreads) void batch_step_kernel(
    const S* __restrict__ src, S* __restrict__ dst, const uint8_t* __restrict__ cls,
    const uint32_t* __restrict__ flags, const StepParams* __restrict__ cells,
    const int* __restrict__ active, const int* __restrict__ list,
    const int* __restrict__ n_list, int nz_cell, long long cell_size, int zper,
    double* __restrict__ partials) {
  using C = typename ComputeOf<S>::type;
  const int zblocks = nz_cell / zper;
  const int slot = blockIdx.z / zblocks;
  const int zb = blockIdx.z - slot * zblocks;  // z block within the cell
  if (list && slot >= *n_list) return;
  const int b = list ? list[slot] : slot;
  if (!active[b]) return;
  const StepParams p = cells[b];
  const long long off = (long long)b * cell_size;
  // cell b's addresses start at off, a whole number of runs: its state
  // starts at kQ * off
  const S* s = src + off * kQ;
  S* d = dst + off * kQ;
  const uint8_t* cl = cls + off;
  const uint32_t* f = flags + off;
  double v[kRedVals] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = 0; i < zper; ++i) {
    const int z = zb * zper + i;
    const TileCell tc = tile_cell(p.t, z);
    const int c = tc.c;
    const uint8_t k = tc.inside ? cl[c] : kClsSolid;
    const bool solid = k & kClsSolid;
    const uint32_t fl = tc.inside ? flag_word(k, f, c) : kSolid;
    const unsigned long long fluid = __ballot(!solid);
    const bool edge_x = __ballot(tc.x == 0 || tc.x == p.nx - 1) != 0;
    if (!solid_stores<S>(p.solid_writes, solid, fluid)) continue;
    S out[kQ];
    C mom[5];
    if (solid)
      solid_node<S>(s, out, p.t, c, fl);
    else
      update_node<S, COLL, WALL, false>(s, out, f, p, tc.x, tc.y, z, c, fl, edge_x, mom);
    if (tc.inside) store_node<S, NT, false>(d, out, p.t, (long long)z * p.t.plane, tc.r);
    if (solid) continue;
    if constexpr (RED) {
      const double rho = mom[0], ux = mom[1], uy = mom[2], uz = mom[3];
      const double u2 = ux * ux + uy * uy + uz * uz;
      v[0] += ux;
      v[1] += uy;
      v[2] += uz;
      v[3] += rho;
      if (isfinite(u2) && isfinite(rho))
        v[4] = fmax(v[4], u2);
      else
        v[5] += 1.0;
    }
  }
  if constexpr (RED) {
    const int kind[kRedVals] = {0, 0, 0, 0, 1, 0, 0, 0};
    const long long blk = blockIdx.x + (long long)gridDim.x * ((long long)b * zblocks + zb);
    block_reduce<kRedVals>(v, kind, partials + blk * kRedVals);
  }
}

// The kernels below (checks, reductions, set-up) are compiled with the host
// code only; the per-storage step translation units define LBM_STEP_TU and
// stop here.
#ifndef LBM_STEP_TU

// Per-cell convergence record, updated on the device at every check.
struct CellStatus {
  double prev_u;   // U_x at the previous check
  double u[3];     // superficial velocity at the last check
  double res;      // relative change of U_x over the last interval
  double max_u2;   // largest |u|^2 at the last check
  long long steps; // steps taken by the cell
  int below;       // consecutive checks below tol
  int status;      // 0 running, 1 converged, 2 unstable, 3 step limit
  int parity;      // buffer holding the cell's final state (when stopped)
  int pad;
};

// One block per cell folds that cell's segment of block partials (fixed
// order) into results[b].
__global__ __launch_bounds__(kRedThreads) void cell_reduce_kernel(const double* __restrict__ partials,
                                                                  long long blocks_per_cell,
                                                                  const int* __restrict__ active,
                                                                  double* __restrict__ results) {
  const int b = blockIdx.x;
  if (!active[b]) return;
  double v[kRedVals] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int kind[kRedVals] = {0, 0, 0, 0, 1, 0, 0, 0};
  const double* in = partials + (long long)b * blocks_per_cell * kRedVals;
  for (long long i = threadIdx.x; i < blocks_per_cell; i += kRedThreads)
#pragma unroll
    for (int j = 0; j < kRedVals; ++j)
      v[j] = kind[j] ? fmax(v[j], in[i * kRedVals + j]) : v[j] + in[i * kRedVals + j];
  block_reduce<kRedVals>(v, kind, results + (long long)b * kRedVals);
}

// Convergence test of every running cell after a check step (one block):
// residual |U - U_prev| / |U| below tol three times in a row -> converged;
// non-finite or |u| above the sound speed -> unstable; step limit -> stop.
// active[b], the running cells in order (list) and their count are
// rewritten.
__global__ __launch_bounds__(1024) void batch_check_kernel(const double* __restrict__ results,
                                                           CellStatus* __restrict__ st,
                                                           int* __restrict__ active,
                                                           int* __restrict__ list,
                                                           int* __restrict__ n_active, int n_cells,
                                                           double inv_cell_size, double tol,
                                                           long long max_steps, int interval,
                                                           int parity_now) {
  __shared__ int count[32];
  __shared__ int base;
  if (threadIdx.x == 0) base = 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  // chunks of blockDim.x cells (every thread runs every chunk, so that the
  // block-wide scans below see all of them)
  for (int b0 = 0; b0 < n_cells; b0 += blockDim.x) {
    const int b = b0 + threadIdx.x;
    int running = 0;
    if (b < n_cells) {
      CellStatus c = st[b];
      if (c.status == 0) {
        c.steps += interval;
        const double* r = results + (long long)b * kRedVals;
        const double U = r[0] * inv_cell_size;
        c.u[0] = U;
        c.u[1] = r[1] * inv_cell_size;
        c.u[2] = r[2] * inv_cell_size;
        c.max_u2 = r[4];
        if (r[5] > 0 || !isfinite(U) || r[4] > 1.0 / 3.0) {
          c.status = 2;
        } else {
          c.res = U != 0.0 ? fabs(U - c.prev_u) / fabs(U) : (U == c.prev_u ? 0.0 : INFINITY);
          c.prev_u = U;
          c.below = c.res < tol ? c.below + 1 : 0;
          if (c.below >= 3) c.status = 1;
          else if (c.steps >= max_steps) c.status = 3;
        }
        if (c.status != 0) c.parity = parity_now;
        st[b] = c;
      }
      active[b] = c.status == 0;
      running = c.status == 0;
    }
    // position of this cell among the chunk's running cells: inclusive scan
    // within the wavefront, then the wavefront totals in order
    int pre = running;
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_up(pre, off, 64);
      if (lane >= off) pre += o;
    }
    if (lane == 63) count[wv] = pre;
    __syncthreads();
    int before = base;
    for (int w = 0; w < wv; ++w) before += count[w];
    if (running) list[before + pre - 1] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = base;
      for (int w = 0; w < nw; ++w) t += count[w];
      base = t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_active = base;
}

// Start of a batch run: every cell running (and listed), counters cleared.
__global__ void batch_reset_kernel(CellStatus* __restrict__ st, int* __restrict__ active,
                                   int* __restrict__ list, int* __restrict__ n_active,
                                   int n_cells, int parity) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0) *n_active = n_cells;
  if (b >= n_cells) return;
  CellStatus c{};
  c.res = INFINITY;
  c.parity = parity;
  st[b] = c;
  active[b] = 1;
  list[b] = b;
}

__global__ void fill_int_kernel(int* __restrict__ a, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// Copy each stopped cell's final state into buffer `to` when it stopped in
// the other buffer (so that the whole batch is read from one buffer).
template <typename S>
__global__ void batch_align_kernel(S* __restrict__ to, const S* __restrict__ from,
                                   const CellStatus* __restrict__ st, int to_parity,
                                   long long cell_size, Tiling t, int n_cells) {
  const long long total = (long long)n_cells * cell_size;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(i / cell_size);
    if (st[b].status == 0 || st[b].parity == to_parity) continue;
#pragma unroll
    for (int k = 0; k < kQ; ++k) to[state_slot<S>(t, k, i)] = from[state_slot<S>(t, k, i)];
  }
}

// Fold n partial vectors into gridDim.x vectors: block b takes a contiguous
// chunk in a fixed order.
__global__ __launch_bounds__(kRedThreads) void reduce_partials_kernel(const double* __restrict__ in,
                                                                      long long n, int max_mask,
                                                                      double* __restrict__ out) {
  double v[kRedVals] = {0, 0, 0, 0, 0, 0, 0, 0};
  int kind[kRedVals];
#pragma unroll
  for (int i = 0; i < kRedVals; ++i) kind[i] = (max_mask >> i) & 1;
  const long long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long long b0 = blockIdx.x * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
  for (long long b = b0 + threadIdx.x; b < b1; b += kRedThreads)
#pragma unroll
    for (int i = 0; i < kRedVals; ++i)
      v[i] = kind[i] ? fmax(v[i], in[b * kRedVals + i]) : v[i] + in[b * kRedVals + i];
  block_reduce<kRedVals>(v, kind, out + (long long)blockIdx.x * kRedVals);
}

template <typename S>
__global__ __launch_bounds__(kRedThreads) void reduce_state_kernel(const S* __restrict__ src,
                                                                   const uint32_t* __restrict__ flags,
                                                                   Tiling t, int naddr,
                                                                   double sigma,
                                                                   double* __restrict__ partials) {
  double v[kRedVals] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long c = blockIdx.x * kRedThreads + threadIdx.x; c < naddr;
       c += (long long)gridDim.x * kRedThreads) {
    if (flags[c] & kSolid) continue;
    double g[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) g[k] = stored_to_g<S>(src[state_slot<S>(t, k, c)], k, sigma);
    double rho, ux, uy, uz;
    moments<double>(g, rho, ux, uy, uz);
    const double u2 = ux * ux + uy * uy + uz * uz;
    v[0] += ux;
    v[1] += uy;
    v[2] += uz;
    v[3] += rho;
    if (isfinite(u2) && isfinite(rho)) {
      v[4] = fmax(v[4], u2);
    } else {
      v[5] += 1.0;
    }
  }
  const int kind[kRedVals] = {0, 0, 0, 0, 1, 0, 0, 0};
  block_reduce<kRedVals>(v, kind, partials + blockIdx.x * kRedVals);
}

// Momentum-exchange force over the wall links (f = g + w), same wall rule as
// the step kernel.  Threads walk the tiled addresses; padding cells are solid.
template <typename S, int WALL>
__global__ __launch_bounds__(kRedThreads) void drag_kernel(const S* __restrict__ src,
                                                           const uint32_t* __restrict__ flags,
                                                           const StepParams p,
                                                           double* __restrict__ partials) {
  double v[kRedVals] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int naddr = p.t.plane * p.nz;
  for (long long cc = blockIdx.x * kRedThreads + threadIdx.x; cc < naddr;
       cc += (long long)gridDim.x * kRedThreads) {
    const int c = (int)cc;
    const uint32_t fl = flags[c];
    if ((fl & kSolid) || !(fl & kLinkMask)) continue;
    int x, y, z;
    p.t.coords(c, x, y, z);
    double m1[4] = {0, 0, 0, 0};
    if constexpr (WALL == kGEN) {
      if (p.wall == kRuleIEBB) {
        double u1[3];
        stored_moments<S, double>(src, p.t, c, m1[0], u1);
        m1[1] = u1[0];
        m1[2] = u1[1];
        m1[3] = u1[2];
      }
    }
    for (int k = 1; k < kQ; ++k) {
      if (!(fl & (1u << k))) continue;
      const int j = kLat.opp[k];
      const double own_j = stored_to_g<S>(src[state_slot<S>(p.t, j, c)], j, p.sigma);
      double back = own_j;
      if constexpr (WALL == kGEN) {
        const int sx = (x - kLat.ex[k] + p.nx) % p.nx, sy = (y - kLat.ey[k] + p.ny) % p.ny,
                  sz = (z - kLat.ez[k] + p.nz) % p.nz;
        const double q = (double)Storage<S>::to_float(src[state_slot<S>(p.t, k, p.t.at(sx, sy, sz))]);
        const FarNode n2 = far_node(p, x, y, z, k, 1);
        back = general_wall_value<S, double>(src, flags, p, x, y, z, c, k, q, fl, m1,
                                             (double)Storage<S>::to_float(src[state_slot<S>(p.t, j, n2.c)]),
                                             (double)Storage<S>::to_float(src[state_slot<S>(p.t, j, c)]),
                                             (double)Storage<S>::to_float(src[state_slot<S>(p.t, k, c)]));
      } else if (WALL == kCLI) {
        const int sx = (x - kLat.ex[k] + p.nx) % p.nx, sy = (y - kLat.ey[k] + p.ny) % p.ny,
                  sz = (z - kLat.ez[k] + p.nz) % p.nz;
        const double a = (double)Storage<S>::to_float(src[state_slot<S>(p.t, k, p.t.at(sx, sy, sz))]);
        const int tx = x + kLat.ex[k];
        const int fx = (tx + p.nx) % p.nx, fy = (y + kLat.ey[k] + p.ny) % p.ny,
                  fz = (z + kLat.ez[k] + p.nz) % p.nz;
        double far_j = stored_to_g<S>(src[state_slot<S>(p.t, j, p.t.at(fx, fy, fz))], j, p.sigma);
        const double jw = kLat.w[k] == 1.0 / 18.0 ? p.jump_axis : p.jump_diag;
        if (tx >= p.nx) far_j -= jw;
        if (tx < 0) far_j += jw;
        back = a * far_j - a * stored_to_g<S>(src[state_slot<S>(p.t, k, c)], k, p.sigma) + own_j;
      }
      const double tot = (own_j + kLat.w[j]) + (back + kLat.w[k]);
      v[0] += kLat.ex[j] * tot;
      v[1] += kLat.ey[j] * tot;
      v[2] += kLat.ez[j] * tot;
    }
  }
  const int kind[kRedVals] = {0, 0, 0, 0, 0, 0, 0, 0};
  block_reduce<kRedVals>(v, kind, partials + blockIdx.x * kRedVals);
}

// Second pass: one block folds the per-block partials in a fixed order.
__global__ __launch_bounds__(kRedThreads) void reduce_final_kernel(const double* __restrict__ partials,
                                                                   int nblocks, int max_mask,
                                                                   double* __restrict__ out) {
  double v[kRedVals] = {0, 0, 0, 0, 0, 0, 0, 0};
  int kind[kRedVals];
#pragma unroll
  for (int i = 0; i < kRedVals; ++i) kind[i] = (max_mask >> i) & 1;
  for (int b = threadIdx.x; b < nblocks; b += kRedThreads)
#pragma unroll
    for (int i = 0; i < kRedVals; ++i)
      v[i] = kind[i] ? fmax(v[i], partials[b * kRedVals + i]) : v[i] + partials[b * kRedVals + i];
  block_reduce<kRedVals>(v, kind, out);
}

// ------------------------------------------------------------ state I/O

template <typename S>
__global__ void fill_kernel(S* __restrict__ buf, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    buf[i] = Storage<S>::from_float(0);
}

// Wall-link coefficients (not scaled) into the solid-source slots of both buffers.
template <typename S>
__global__ void scatter_kernel(S* __restrict__ a, S* __restrict__ b,
                               const long long* __restrict__ slot,
                               const double* __restrict__ value, long long n) {
  using C = typename Storage<S>::compute;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const S v = Storage<S>::from_float((C)value[i]);
    a[slot[i]] = v;
    b[slot[i]] = v;
  }
}

// Host-facing arrays are in row-major cell order (index c = x + nx (y + ny z)
// within a z period of nz_cell planes; batches stack such periods); the
// device buffers are in tiled order.  addr_of maps one to the other.
__device__ __forceinline__ int addr_of(const Tiling& t, long long c, long long cell_cells,
                                       int cell_addrs) {
  const long long b = c / cell_cells;
  return (int)(b * cell_addrs) + t.from_linear(c - b * cell_cells);
}

// Direction k, cells [c0, c0 + n) in row-major order, to/from a
// double staging buffer (values are g_k; 16-bit storage is decoded / encoded
// with sigma).
template <typename S>
__global__ void get_plane_kernel(const S* __restrict__ buf, const uint32_t* __restrict__ flags,
                                 Tiling t, long long cell_cells, int cell_addrs, int k,
                                 double sigma, int c0, int n, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = addr_of(t, c0 + i, cell_cells, cell_addrs);
  out[i] = (flags[a] & kSolid) ? 0.0 : stored_to_g<S>(buf[state_slot<S>(t, k, a)], k, sigma);
}

template <typename S>
__global__ void set_plane_kernel(S* __restrict__ buf, const uint32_t* __restrict__ flags,
                                 Tiling t, long long cell_cells, int cell_addrs, int k,
                                 double sigma, int c0, int n, const double* __restrict__ in) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = addr_of(t, c0 + i, cell_cells, cell_addrs);
  if (!(flags[a] & kSolid)) buf[state_slot<S>(t, k, a)] = g_to_stored<S>(in[i], k, sigma);
}

// g = g^eq(drho, u) for fluid cells [c0, c0 + n) (row-major order); stage =
// drho | ux | uy | uz blocks of n doubles (all-zero staging gives the rest
// state).
template <typename S>
__global__ void init_eq_kernel(S* __restrict__ buf, const uint32_t* __restrict__ flags,
                               Tiling t, long long cell_cells, int cell_addrs,
                               double sigma, int c0, int n,
                               const double* __restrict__ stage) {
  using C = typename ComputeOf<S>::type;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = addr_of(t, c0 + i, cell_cells, cell_addrs);
  if (flags[c] & kSolid) return;
  const C rho = (C)stage[i], ux = (C)stage[n + i], uy = (C)stage[2 * n + i],
          uz = (C)stage[3 * n + i];
  const C usq = ux * ux + uy * uy + uz * uz;
  C g[kQ];
#define LBM_EQ(K) g[K] = geq<C, K>(rho, ux, uy, uz, usq);
  LBM_EQ(0) LBM_EQ(1) LBM_EQ(2) LBM_EQ(3) LBM_EQ(4) LBM_EQ(5) LBM_EQ(6) LBM_EQ(7) LBM_EQ(8)
  LBM_EQ(9) LBM_EQ(10) LBM_EQ(11) LBM_EQ(12) LBM_EQ(13) LBM_EQ(14) LBM_EQ(15) LBM_EQ(16)
  LBM_EQ(17) LBM_EQ(18)
#undef LBM_EQ
#pragma unroll
  for (int k = 0; k < kQ; ++k) buf[state_slot<S>(t, k, c)] = g_to_stored<S>((double)g[k], k, sigma);
}

// drho, u of cells [c0, c0 + n) (row-major order) into stage (drho | ux |
// uy | uz blocks).
template <typename S>
__global__ void macro_kernel(const S* __restrict__ buf, const uint32_t* __restrict__ flags,
                             Tiling t, long long cell_cells, int cell_addrs,
                             double sigma, int c0, int n, double* __restrict__ stage) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = addr_of(t, c0 + i, cell_cells, cell_addrs);
  double rho = 0, ux = 0, uy = 0, uz = 0;
  if (!(flags[c] & kSolid)) {
    double g[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) g[k] = stored_to_g<S>(buf[state_slot<S>(t, k, c)], k, sigma);
    moments<double>(g, rho, ux, uy, uz);
  }
  stage[i] = rho;
  stage[n + i] = ux;
  stage[2 * n + i] = uy;
  stage[3 * n + i] = uz;
}

// Multiply the stored values of fluid cells by a power of two (exact unless
// a value leaves the normal range); used to move the 16-bit storage scale.
template <typename S>
__global__ void rescale_kernel(S* __restrict__ buf, const uint32_t* __restrict__ flags,
                               Tiling t, int naddr, float factor) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < naddr;
       c += (long long)gridDim.x * blockDim.x) {
    if (flags[c] & kSolid) continue;
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
      S* q = buf + state_slot<S>(t, k, c);
      *q = Storage<S>::from_float(Storage<S>::to_float(*q) * factor);
    }
  }
}

// IEBB's side buffer for a state set from outside the time loop: the
// velocity of every near-wall cell from its stored values.
template <typename S>
__global__ void side_moments_kernel(const S* __restrict__ buf, const uint8_t* __restrict__ cls,
                                    Tiling t, int naddr, void* side) {
  using C = typename ComputeOf<S>::type;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < naddr;
       c += (long long)gridDim.x * blockDim.x) {
    if ((cls[c] & (kClsNearWall | kClsSolid)) != kClsNearWall) continue;
    C d, u[3];
    stored_moments<S, C>(buf, t, (int)c, d, u);
    C* o = static_cast<C*>(side) + 4 * c;
    o[0] = u[0];
    o[1] = u[1];
    o[2] = u[2];
  }
}

#endif  // LBM_STEP_TU

}  // namespace lbm
