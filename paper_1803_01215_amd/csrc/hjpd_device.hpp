// Device-side helpers shared by the hjpd kernels (gfx950, wave64).
//
//  - the counter-based random start (section 6 set-up: every free coordinate
//    of x_j starts within 0.1 of the query point, every multiplier within 0.1
//    of 0): SplitMix64 (Steele, Lea, Flood 2014) evaluated at a counter built
//    from (point, array, node, coordinate);
//  - lane-group primitives: a query point is owned by a group of L
//    consecutive lanes of a wavefront, each lane holding K consecutive time
//    nodes, so the difference operator D (Appendix A.1.1: (Dz)_j = z_j -
//    z_{j-1}, (D^T p)_j = p_j - p_{j+1}) needs one neighbour exchange per
//    direction per iteration, done with DPP wavefront shifts;
//  - precision-generic math wrappers (float: hardware transcendental and
//    reciprocal instructions; double: OCML).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hjpd {

enum : int { kArrX = 0, kArrP = 1, kArrY = 2, kArrQ = 3 };
enum : int { kConverged = 0, kMaxIter = 1, kNonFinite = 2, kBadInput = 3, kValueStalled = 4 };

// ---------------------------------------------------------------------------
// Random start
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t sm64_finalize(uint64_t s) {
  // SplitMix64 output mix: two xor-shift-multiply rounds and a final xor-shift.
  s ^= s >> 30;
  s *= 0xBF58476D1CE4E5B9ull;
  s ^= s >> 27;
  s *= 0x94D049BB133111EBull;
  return s ^ (s >> 31);
}

// Uniform perturbation in [-0.1, 0.1) for (point, array, node, coordinate):
// output number c+1 of the SplitMix64 sequence whose state starts at `seed`
// (state after c+1 steps = seed + (c+1) * golden-ratio increment), top 53
// bits as a double in [0,1), mapped affinely.
__device__ __forceinline__ double start_noise(uint64_t seed, uint64_t point, int arr, int node, int coord) {
  const uint64_t ctr = (point << 22) | (uint64_t(arr) << 20) | (uint64_t(node) << 10) | uint64_t(coord);
  const uint64_t bits = sm64_finalize(seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull);
  const double u = __dmul_rn(double(bits >> 11), 0x1.0p-53);
  return __dsub_rn(__dmul_rn(0.2, u), 0.1);
}

// ---------------------------------------------------------------------------
// Math wrappers
// ---------------------------------------------------------------------------

template <typename T> struct M;

template <> struct M<float> {
  static __device__ __forceinline__ void sincos(float a, float* s, float* c) { __sincosf(a, s, c); }
  static __device__ __forceinline__ float sqrt(float a) { return __builtin_sqrtf(a); }
  static __device__ __forceinline__ float rsqrt(float a) { return __frsqrt_rn(a); }
  static __device__ __forceinline__ float rcp(float a) { return __builtin_amdgcn_rcpf(a); }
  static __device__ __forceinline__ float tanh(float a) { return ::tanhf(a); }
  static __device__ __forceinline__ float exp(float a) { return ::expf(a); }
  static __device__ __forceinline__ float fmax(float a, float b) { return ::fmaxf(a, b); }
  static __device__ __forceinline__ float fabs_(float a) { return ::fabsf(a); }
  static __device__ __forceinline__ bool finite(float a) { return __builtin_isfinite(a); }
  // Quotient and square root inside the iteration: the hardware reciprocal
  // and square root (about 1 ulp) instead of the correctly rounded sequences
  // (about ten instructions each, with a branch for the quotient).  FP32
  // results move by rounding only.
  static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
  static __device__ __forceinline__ float sqrt_fast(float a) { return __builtin_amdgcn_sqrtf(a); }
};

template <> struct M<double> {
  static __device__ __forceinline__ void sincos(double a, double* s, double* c) { ::sincos(a, s, c); }
  static __device__ __forceinline__ double sqrt(double a) { return ::sqrt(a); }
  static __device__ __forceinline__ double rsqrt(double a) { return ::rsqrt(a); }
  static __device__ __forceinline__ double rcp(double a) { return 1.0 / a; }
  static __device__ __forceinline__ double tanh(double a) { return ::tanh(a); }
  static __device__ __forceinline__ double exp(double a) { return ::exp(a); }
  static __device__ __forceinline__ double fmax(double a, double b) { return ::fmax(a, b); }
  static __device__ __forceinline__ double fabs_(double a) { return ::fabs(a); }
  static __device__ __forceinline__ bool finite(double a) { return __builtin_isfinite(a); }
  static __device__ __forceinline__ double div(double a, double b) { return a / b; }
  static __device__ __forceinline__ double sqrt_fast(double a) { return ::sqrt(a); }
};

// ---------------------------------------------------------------------------
// Cross-lane movement.  DPP wavefront shifts (GFX9-family controls kept by
// CDNA): wave_shr:1 gives lane i the value of lane i-1, wave_shl:1 gives lane i
// the value of lane i+1.  Edge lanes receive 0 and are overwritten by the
// caller (group boundaries use their own data).
// ---------------------------------------------------------------------------

// bound_ctrl set: the lane without a source (lane 0 for wave_shr, lane 63 for
// wave_shl) reads 0, so no register has to be cleared first.
__device__ __forceinline__ int dpp_from_prev(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true);  // wave_shr:1
}
__device__ __forceinline__ int dpp_from_next(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true);  // wave_shl:1
}

__device__ __forceinline__ float from_prev(float v) {
  return __builtin_bit_cast(float, dpp_from_prev(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float from_next(float v) {
  return __builtin_bit_cast(float, dpp_from_next(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double from_prev(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = uint32_t(dpp_from_prev(int(uint32_t(b))));
  const uint32_t hi = uint32_t(dpp_from_prev(int(uint32_t(b >> 32))));
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}
__device__ __forceinline__ double from_next(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = uint32_t(dpp_from_next(int(uint32_t(b))));
  const uint32_t hi = uint32_t(dpp_from_next(int(uint32_t(b >> 32))));
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

// DPP controls used below (GFX9 family, kept by CDNA):
//   row_shr:1 / row_shl:1   lane i of a 16-lane row reads lane i-1 / i+1 of the
//                           same row; the row's first / last lane reads 0
//                           (bound_ctrl set);
//   quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror (lane i of each
//   8-lane half reads lane 7-i), row_mirror (lane i of a row reads lane 15-i):
//   the four exchanges of a 16-lane butterfly all-reduce.
enum : int { kDppRowShl1 = 0x101, kDppRowShr1 = 0x111, kDppQuad1032 = 0xB1, kDppQuad2301 = 0x4E,
             kDppRowHalfMirror = 0x141, kDppRowMirror = 0x140 };

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b)), CTRL, 0xf, 0xf, true));
  const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b >> 32)), CTRL, 0xf, 0xf, true));
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

// Value of v held by the previous lane of the group (lane l-1 of an aligned
// group of L lanes); the group's first lane (l = 0) gets 0.
template <int L, typename T>
__device__ __forceinline__ T group_prev0(T v, int l) {
  if constexpr (L >= 32) {
    const T s = from_prev(v);
    return (l == 0) ? T(0) : s;
  } else {
    const T s = dpp_f<kDppRowShr1>(v);  // row start reads 0
    if constexpr (L == 16) return s;
    else return (l == 0) ? T(0) : s;
  }
}

// Value of v held by the previous lane of the group, and `fill` in the
// group's first lane (fill must be 0 in every other lane).  One select (or
// one add for 16-lane groups, whose row shift already reads 0 there).
template <int L, typename T>
__device__ __forceinline__ T group_prev_fill(T v, int l, T fill) {
  if constexpr (L >= 32) {
    const T s = from_prev(v);
    return (l == 0) ? fill : s;
  } else {
    const T s = dpp_f<kDppRowShr1>(v);  // row start reads 0
    if constexpr (L == 16) return s + fill;
    else return (l == 0) ? fill : s;
  }
}

// Value of v held by the next lane of the group; the group's last lane gets 0.
template <int L, typename T>
__device__ __forceinline__ T group_next0(T v, int l) {
  if constexpr (L >= 32) {
    const T s = from_next(v);
    return (l == L - 1) ? T(0) : s;
  } else {
    const T s = dpp_f<kDppRowShl1>(v);  // row end reads 0
    if constexpr (L == 16) return s;
    else return (l == L - 1) ? T(0) : s;
  }
}

// Sum over the L lanes of an aligned group (L a power of two <= 64); every
// lane of the group receives the same total (each exchange adds a pair in
// both lanes, and addition commutes).  Within a 16-lane row: DPP butterfly;
// across rows: xor shuffles.
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v) {
  if constexpr (L >= 2) v += dpp_f<kDppQuad1032>(v);
  if constexpr (L >= 4) v += dpp_f<kDppQuad2301>(v);
  if constexpr (L >= 8) v += dpp_f<kDppRowHalfMirror>(v);
  if constexpr (L >= 16) v += dpp_f<kDppRowMirror>(v);
  if constexpr (L >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (L >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

template <int L>
__device__ __forceinline__ int group_or(int v) {
#pragma unroll
  for (int m = 1; m < L; m <<= 1) v |= __shfl_xor(v, m, 64);
  return v;
}

}  // namespace hjpd
