// Device building blocks shared by the library's kernels: the counter-based random numbers of
// the common-random-numbers contract, and workgroup reductions and scans for 64-lane waves.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc2 {

// Random streams of the counter contract: counter word 3 = (k << 8) | stream.
enum : uint32_t {
  kStreamInit = 1,      // x_0 normals, per particle slot
  kStreamStep = 2,      // propagation normals, per particle slot, index (t-1)*d + q
  kStreamResample = 3,  // resampling uniforms: systematic one per filter (slot word all ones),
                        // multinomial one per offspring slot; index t-1
  kStreamPrior = 4,     // theta_1 ~ prior, per sample, iteration 1
  kStreamMove = 5,      // Langevin / random-walk move normals, per sample
  kStreamOuter = 6      // outer systematic resampling uniform, per series
};
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kHalfLog2Pi = 0.91893853320467274178032973640562;

__device__ __forceinline__ uint32_t stream_word(uint32_t k, uint32_t stream) {
  return (k << 8) | stream;
}

// a ^ b ^ c in one instruction: gfx950's three-input bitwise operation, whose 8-bit table is
// indexed by the bits of (a, b, c) as (0xF0, 0xCC, 0xAA); 0xF0 ^ 0xCC ^ 0xAA = 0x96.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds; in each, words 0 and 2 are
// multiplied (32x32 -> 64) by the two round multipliers, the high halves are mixed with words
// 1 and 3 and the round key, and the key advances by the Weyl constants.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint64_t seed) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  // An empty statement that the compiler must assume changes the key: it then advances the key
  // schedule (two scalar adds per round) inside every call instead of holding all twenty round
  // keys in scalar registers for the whole kernel, which spilled scalar registers into vector
  // lanes and cost the filter kernel up to a quarter of its time.  The seed is a kernel argument,
  // uniform across the wave, which the scalar-register constraint requires.
  asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// NB Philox4x32-10 blocks that differ only in the first counter word, run under one key
// schedule (the same numbers as NB calls of philox4x32_10, with the scalar key advance shared).
template <int NB>
__device__ __forceinline__ void philox4x32_10_n(const uint32_t (&c0)[NB], uint32_t c1,
                                                uint32_t c2, uint32_t c3, uint64_t seed,
                                                uint4 (&out)[NB]) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  asm volatile("" : "+s"(k0), "+s"(k1));  // as in philox4x32_10
  uint32_t a[NB], b[NB], c[NB], d[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    a[i] = c0[i];
    b[i] = c1;
    c[i] = c2;
    d[i] = c3;
  }
#pragma unroll
  for (int r = 0; r < 10; ++r) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)a[i];
      const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[i];
      const uint32_t n0 = xor3((uint32_t)(p1 >> 32), b[i], k0);
      const uint32_t n2 = xor3((uint32_t)(p0 >> 32), d[i], k1);
      b[i] = (uint32_t)p1;
      d[i] = (uint32_t)p0;
      a[i] = n0;
      c[i] = n2;
    }
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) out[i] = make_uint4(a[i], b[i], c[i], d[i]);
}

// Box-Muller (Box & Muller 1958) on one word pair: u1 = (wa + 1) 2^-32 in (0, 1],
// u2 = wb 2^-32 in [0, 1); z0 = r cos(2 pi u2), z1 = r sin(2 pi u2), r = sqrt(-2 ln u1).
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double &z0, double &z1) {
  const double u1 = ((double)wa + 1.0) * 0x1p-32;
  const double u2 = (double)wb * 0x1p-32;
  const double r = sqrt(-2.0 * log(u1));
  double s, c;
  sincos(kTwoPi * u2, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

// The FP32 form runs the transcendentals on the hardware units: v_log_f32 is log2, v_sqrt_f32,
// and v_sin_f32 / v_cos_f32 take their argument in revolutions, so cos(2 pi u2) is one
// instruction.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float &z0, float &z1) {
  const float u1 = ((float)wa + 1.0f) * 0x1p-32f;
  const float u2 = (float)wb * 0x1p-32f;
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
  z0 = r * __builtin_amdgcn_cosf(u2);
  z1 = r * __builtin_amdgcn_sinf(u2);
}

// exp and reciprocal in the arithmetic type: library FP64, hardware FP32 (v_exp_f32 is 2^x).
__device__ __forceinline__ double fexp(double x) { return exp(x); }
__device__ __forceinline__ float fexp(float x) {
  return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
}
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// The four normals of one Philox block (pairs 2b and 2b+1 of the stream).
template <typename R>
__device__ __forceinline__ void normals4(uint32_t c0, uint32_t block, uint32_t c2, uint32_t c3,
                                         uint64_t seed, R z[4]) {
  const uint4 w = philox4x32_10(c0, block, c2, c3, seed);
  box_muller(w.x, w.y, z[0], z[1]);
  box_muller(w.z, w.w, z[2], z[3]);
}

// Normal number n of a stream (pair n/2 in block n/4).
template <typename R>
__device__ __forceinline__ R normal_n(uint32_t c0, uint32_t c2, uint32_t c3, uint32_t n,
                                      uint64_t seed) {
  const uint32_t p = n >> 1;
  const uint4 w = philox4x32_10(c0, p >> 1, c2, c3, seed);
  R z0, z1;
  if (p & 1u)
    box_muller(w.z, w.w, z0, z1);
  else
    box_muller(w.x, w.y, z0, z1);
  return (n & 1u) ? z1 : z0;
}

// Uniform number m in (0, 1] of a stream: block m/4, word m%4, (w + 1) 2^-32 (exact in FP64).
__device__ __forceinline__ double uniform_m(uint32_t c0, uint32_t c2, uint32_t c3, uint32_t m,
                                            uint64_t seed) {
  const uint4 w = philox4x32_10(c0, m >> 2, c2, c3, seed);
  const uint32_t q = m & 3u;
  const uint32_t v = q == 0 ? w.x : q == 1 ? w.y : q == 2 ? w.z : w.w;
  return ((double)v + 1.0) * 0x1p-32;
}

// ---- a lane's run of particle slots in HBM ------------------------------------------------------
// A lane owns N consecutive slots of every per-particle row; the run starts at a multiple of its
// own size in bytes, so it moves with the widest aligned vector accesses.
template <int N, typename T>
__device__ __forceinline__ void store_run(T *dst, const T (&v)[N]) {
  constexpr int B = N * (int)sizeof(T);
  if constexpr (B % 16 == 0) {
#pragma unroll
    for (int b = 0; b < B / 16; ++b) {
      uint4 w;
      __builtin_memcpy(&w, reinterpret_cast<const char *>(v) + 16 * b, 16);
      reinterpret_cast<uint4 *>(dst)[b] = w;
    }
  } else if constexpr (B % 8 == 0) {
#pragma unroll
    for (int b = 0; b < B / 8; ++b) {
      uint2 w;
      __builtin_memcpy(&w, reinterpret_cast<const char *>(v) + 8 * b, 8);
      reinterpret_cast<uint2 *>(dst)[b] = w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) dst[i] = v[i];
  }
}

template <int N, typename T>
__device__ __forceinline__ void load_run(const T *src, T (&v)[N]) {
  constexpr int B = N * (int)sizeof(T);
  if constexpr (B % 16 == 0) {
#pragma unroll
    for (int b = 0; b < B / 16; ++b) {
      const uint4 w = reinterpret_cast<const uint4 *>(src)[b];
      __builtin_memcpy(reinterpret_cast<char *>(v) + 16 * b, &w, 16);
    }
  } else if constexpr (B % 8 == 0) {
#pragma unroll
    for (int b = 0; b < B / 8; ++b) {
      const uint2 w = reinterpret_cast<const uint2 *>(src)[b];
      __builtin_memcpy(reinterpret_cast<char *>(v) + 8 * b, &w, 8);
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = src[i];
  }
}

// component q of a lane's particles, as a run
template <int N, int DX, typename T>
__device__ __forceinline__ void store_comp(T *dst, const T (&v)[N][DX], int q) {
  T r[N];
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = v[i][q];
  store_run<N>(dst, r);
}

template <int N, int DX, typename T>
__device__ __forceinline__ void load_comp(const T *src, T (&v)[N][DX], int q) {
  T r[N];
  load_run<N>(src, r);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i][q] = r[i];
}

// The wave's index in the workgroup as a scalar that the compiler cannot see through: the
// per-wave conditions formed from it inside a loop (w == wid, w < wid for every wave w) are then
// formed where used instead of being hoisted out of the loop and held in registers.
__device__ __forceinline__ int wave_id_opaque() {
  int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  asm volatile("" : "+s"(w));
  return w;
}

// ---- wave and workgroup reductions ------------------------------------------------------------
// Cross-lane moves use the data-parallel (DPP) modifiers of GFX9 VALU instructions instead of
// LDS permutes: quad swaps and row mirrors for butterflies inside each row of 16 lanes, row
// shifts and row broadcasts for scans.  Butterflies combine the same two operands in every lane
// (addition is commutative), so each row ends with bit-identical values; the four row results
// are then combined in a fixed order, either read as scalars or by two row broadcasts into lane
// 63, which is then read, so the wave result is uniform.  Where the lanes a move leaves out take
// the operation's identity, the move folds into the operation (one instruction per stage).  The
// cross-wave stage reads the per-wave values in wave order, so the workgroup result is also
// identical in every thread, which keeps data-dependent branches uniform.  Every lane of the
// wave must be active.
enum : int {
  kDppQuadXor1 = 0xB1,       // quad_perm [1,0,3,2]
  kDppQuadXor2 = 0x4E,       // quad_perm [2,3,0,1]
  kDppRowShr1 = 0x111,       // row_shr:n = 0x110 + n (lanes below n in a row keep `old`)
  kDppRowShr2 = 0x112,
  kDppRowShr4 = 0x114,
  kDppRowShr8 = 0x118,
  kDppRowMirror = 0x140,     // lane 15 - i of the row
  kDppRowHalfMirror = 0x141, // lane 7 - i of the half row
  kDppRowBcast15 = 0x142,    // lane 15 of each row to the next row
  kDppRowBcast31 = 0x143,    // lane 31 to rows 2 and 3
  kDppWaveShr1 = 0x138       // lane i - 1 of the wave (lane 0 keeps `old`)
};

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ int dpp_i32(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROW_MASK, 0xF, false);
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_f64(double old, double v) {
  const uint64_t o = (uint64_t)__double_as_longlong(old), x = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)dpp_i32<CTRL, ROW_MASK>((int)(uint32_t)o, (int)(uint32_t)x);
  const uint32_t hi =
      (uint32_t)dpp_i32<CTRL, ROW_MASK>((int)(uint32_t)(o >> 32), (int)(uint32_t)(x >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t x = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64<kDppQuadXor1>(v, v));
  v = fmax(v, dpp_f64<kDppQuadXor2>(v, v));
  v = fmax(v, dpp_f64<kDppRowHalfMirror>(v, v));
  v = fmax(v, dpp_f64<kDppRowMirror>(v, v));
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)),
              fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// The FP32 maximum over a wave (exact, like any maximum: converting it to FP64 afterwards gives
// the FP64 maximum of the converted values).
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(dpp_i32<CTRL>(__float_as_int(v), __float_as_int(v)));
}

__device__ __forceinline__ float readlane_f32(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// A lane's value in the arithmetic type (lane index uniform across the wave).
__device__ __forceinline__ float readlane_r(float v, int lane) { return readlane_f32(v, lane); }
__device__ __forceinline__ double readlane_r(double v, int lane) { return readlane_f64(v, lane); }

// The FP32 maximum of a wave, taken on order-preserving integer keys of the values (the bits,
// with the magnitude bits of negative values flipped), which orders every non-NaN float as a
// signed integer: an integer maximum takes its cross-lane operand straight from the DPP modifier,
// where a floating-point one would first quiet it.  The row results are combined inside the
// wave by row broadcasts, and lane 63 holds the maximum.
__device__ __forceinline__ int fkey(float v) {
  const int b = __float_as_int(v);
  return b ^ ((b >> 31) & 0x7FFFFFFF);
}
__device__ __forceinline__ float wave_max(float v) {
  // the fill of lanes a move leaves out is INT_MIN, the identity of the maximum
  constexpr int kLo = (int)0x80000000u;
  int k = fkey(v);
  k = max(k, __builtin_amdgcn_update_dpp(kLo, k, kDppQuadXor1, 0xF, 0xF, false));
  k = max(k, __builtin_amdgcn_update_dpp(kLo, k, kDppQuadXor2, 0xF, 0xF, false));
  k = max(k, __builtin_amdgcn_update_dpp(kLo, k, kDppRowHalfMirror, 0xF, 0xF, false));
  k = max(k, __builtin_amdgcn_update_dpp(kLo, k, kDppRowMirror, 0xF, 0xF, false));
  k = max(k, __builtin_amdgcn_update_dpp(kLo, k, kDppRowBcast15, 0xA, 0xF, false));
  k = max(k, __builtin_amdgcn_update_dpp(kLo, k, kDppRowBcast31, 0xC, 0xF, false));
  const int m = __builtin_amdgcn_readlane(k, 63);
  return __int_as_float(m ^ ((m >> 31) & 0x7FFFFFFF));
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<kDppQuadXor1>(0.0, v);
  v += dpp_f64<kDppQuadXor2>(0.0, v);
  v += dpp_f64<kDppRowHalfMirror>(0.0, v);
  v += dpp_f64<kDppRowMirror>(0.0, v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// The FP32 sum over a wave (the mixed form's sum of squared weights, which only decides whether
// to resample).
// The cross-lane operand with 0, the identity of the sum, where a move leaves a lane out, so that
// the moves fold into the additions.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp0_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF,
                                                    ROW_MASK == 0xF));
}

__device__ __forceinline__ float wave_sum(float v) {
  v += dpp0_f32<kDppQuadXor1>(v);
  v += dpp0_f32<kDppQuadXor2>(v);
  v += dpp0_f32<kDppRowHalfMirror>(v);
  v += dpp0_f32<kDppRowMirror>(v);
  // rows 1 and 3 add rows 0 and 2, then row 3 adds row 1: (r0 + r1) + (r2 + r3) in lane 63, the
  // order of the four row sums as before
  v += dpp0_f32<kDppRowBcast15, 0xA>(v);
  v += dpp0_f32<kDppRowBcast31, 0xC>(v);
  return readlane_f32(v, 63);
}

// Inclusive prefix sum over the 64 lanes of a wave (lane order).
__device__ __forceinline__ double wave_inclusive_sum(double v) {
  v += dpp_f64<kDppRowShr1>(0.0, v);
  v += dpp_f64<kDppRowShr2>(0.0, v);
  v += dpp_f64<kDppRowShr4>(0.0, v);
  v += dpp_f64<kDppRowShr8>(0.0, v);
  v += dpp_f64<kDppRowBcast15, 0xA>(0.0, v);
  v += dpp_f64<kDppRowBcast31, 0xC>(0.0, v);
  return v;
}

// Inclusive prefix maximum over the 64 lanes of a wave (lane order); values are >= -1.
__device__ __forceinline__ int wave_inclusive_max(int v) {
  v = max(v, dpp_i32<kDppRowShr1>(-1, v));
  v = max(v, dpp_i32<kDppRowShr2>(-1, v));
  v = max(v, dpp_i32<kDppRowShr4>(-1, v));
  v = max(v, dpp_i32<kDppRowShr8>(-1, v));
  v = max(v, dpp_i32<kDppRowBcast15, 0xA>(-1, v));
  v = max(v, dpp_i32<kDppRowBcast31, 0xC>(-1, v));
  return v;
}

template <int WAVES>
__device__ __forceinline__ double block_max(double v, double *red) {
  v = wave_max(v);
  if constexpr (WAVES > 1) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    v = red[0];
#pragma unroll
    for (int w = 1; w < WAVES; ++w) v = fmax(v, red[w]);
  }
  return v;
}

template <int WAVES>
__device__ __forceinline__ void block_sum2(double &a, double &b, double *red) {
  a = wave_sum(a);
  b = wave_sum(b);
  if constexpr (WAVES > 1) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
      red[2 * wid] = a;
      red[2 * wid + 1] = b;
    }
    __syncthreads();
    a = red[0];
    b = red[1];
#pragma unroll
    for (int w = 1; w < WAVES; ++w) {
      a += red[2 * w];
      b += red[2 * w + 1];
    }
  }
}

// Sum of D values per thread over the workgroup (D <= 64), delivered to thread p for value p
// (0 in the other threads): the waves' sums are added in wave order, as in block_sum_vec.  A
// thread adds one column only, so the workgroup does not hold every total in every thread.
template <int WAVES, int D>
__device__ __forceinline__ double block_sum_to_thread(double *v, double *red) {
#pragma unroll
  for (int p = 0; p < D; ++p) v[p] = wave_sum(v[p]);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int p = 0; p < D; ++p) red[wid * D + p] = v[p];
  __syncthreads();
  double r = 0.0;
  if (tid < D) {
    r = red[tid];
    for (int w = 1; w < WAVES; ++w) r += red[w * D + tid];
  }
  return r;
}

// Sum of D values per thread over the workgroup (D <= 32); result valid in every thread.
template <int WAVES, int D>
__device__ __forceinline__ void block_sum_vec(double *v, double *red) {
#pragma unroll
  for (int p = 0; p < D; ++p) v[p] = wave_sum(v[p]);
  if constexpr (WAVES > 1) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int p = 0; p < D; ++p) red[wid * D + p] = v[p];
    __syncthreads();
#pragma unroll
    for (int p = 0; p < D; ++p) {
      double s = red[p];
      for (int w = 1; w < WAVES; ++w) s += red[w * D + p];
      v[p] = s;
    }
  }
}

// Exclusive scan over the workgroup of one value per thread (thread order); returns the
// exclusive prefix and sets `total` (identical in all threads).
template <int WAVES>
__device__ __forceinline__ double block_exclusive_scan(double v, double *wsum, double &total) {
  const int lane = threadIdx.x & 63, wid = wave_id_opaque();
  const double inc = wave_inclusive_sum(v);
  const double exc = dpp_f64<kDppWaveShr1>(0.0, inc);
  const double wtot = readlane_f64(inc, 63);
  if constexpr (WAVES == 1) {
    total = wtot;
    return exc;
  } else {
    if (lane == 0) wsum[wid] = wtot;
    __syncthreads();
    double off = 0.0, tot = 0.0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      const double s = wsum[w];
      if (w < wid) off += s;
      tot += s;
    }
    total = tot;
    return off + exc;
  }
}

// Exclusive max-scan over the workgroup of one int (>= -1) per thread (thread order); -1 for
// thread 0.
template <int WAVES>
__device__ __forceinline__ int block_exclusive_max_scan(int v, int *wmax) {
  const int lane = threadIdx.x & 63, wid = wave_id_opaque();
  const int inc = wave_inclusive_max(v);
  int exc = dpp_i32<kDppWaveShr1>(-1, inc);
  if constexpr (WAVES > 1) {
    if (lane == 0) wmax[wid] = __builtin_amdgcn_readlane(inc, 63);
    __syncthreads();
#pragma unroll
    for (int w = 0; w < WAVES; ++w)
      if (w < wid) exc = max(exc, wmax[w]);
  }
  return exc;
}

// Number of entries of the non-decreasing array P[0..n) that are < target, i.e. the lower
// bound of target; fixed trip count for uniform control flow.
__device__ __forceinline__ int lower_bound_lds(const double *P, int n, double target) {
  int pos = 0;
  int step = 1;
  while ((step << 1) <= n) step <<= 1;
  for (; step > 0; step >>= 1) {
    const int probe = pos + step;
    if (probe <= n && P[probe - 1] < target) pos = probe;
  }
  return pos;
}

}  // namespace smc2
