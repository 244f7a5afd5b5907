// Device-side building blocks shared by the kernels of libpsfdecorr (gfx950).
//
// Phase factors exp(2 pi i theta) with theta in turns: theta is formed in
// FP64 (u' x reaches tens of turns, u l0 thousands) and reduced to a
// fraction of a turn in FP64; only the reduced angle goes to FP32.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace psf {

constexpr double kCLight = 299792458.0;      // m/s
constexpr double kInvCLight = 1.0 / 299792458.0;

struct cf32 { float re, im; };

__device__ __forceinline__ cf32 cmul(cf32 a, cf32 b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cf32 conj(cf32 a) { return {a.re, -a.im}; }

// exp(2 pi i theta) for theta in turns, with the hardware sine and cosine:
// the argument reduced to [-1/2, 1/2] turns in FP64, then v_sin / v_cos,
// which take turns (about 4e-7 absolute error).  sin(0) = 0 and cos(0) = 1
// exactly.  For values used once (a sample's phase factor, a row seed); a
// factor raised to powers uses the polynomial form below.
__device__ __forceinline__ cf32 expi_turns_hw(double theta) {
  const float x = static_cast<float>(theta - rint(theta));
  cf32 z;
  z.re = __builtin_amdgcn_cosf(x);
  z.im = __builtin_amdgcn_sinf(x);
  return z;
}

// exp(2 pi i theta) for theta in turns.
//
// FP64 step: q = nearest quarter turn, r = theta - q/4 with |r| <= 1/8 turn
// (q/4 is exact, so r carries the full FP64 accuracy of theta's fraction).
// FP32 step: x = 2 pi r in [-pi/4, pi/4]; sin and cos from their Taylor
// series through x^9 and x^10 (truncation below 2e-9, under FP32 rounding);
// the quadrant q mod 4 rotates (cos, sin) by multiples of 90 degrees.
__device__ __forceinline__ cf32 expi_turns(double theta) {
  const double q = rint(4.0 * theta);
  const double r = fma(-0.25, q, theta);
  const float x = static_cast<float>(r * 6.283185307179586);
  const float x2 = x * x;
  // coefficients (-1)^n / (2n+1)! and (-1)^n / (2n)!
  constexpr float s3 = -1.0f / 6.0f, s5 = 1.0f / 120.0f, s7 = -1.0f / 5040.0f, s9 = 1.0f / 362880.0f;
  constexpr float c2 = -0.5f, c4 = 1.0f / 24.0f, c6 = -1.0f / 720.0f, c8 = 1.0f / 40320.0f,
                  c10 = -1.0f / 3628800.0f;
  const float s = x * (1.0f + x2 * (s3 + x2 * (s5 + x2 * (s7 + x2 * s9))));
  const float c = 1.0f + x2 * (c2 + x2 * (c4 + x2 * (c6 + x2 * (c8 + x2 * c10))));
  const int quad = static_cast<int>(static_cast<long long>(q) & 3);
  cf32 z;
  z.re = (quad == 0) ? c : (quad == 1) ? -s : (quad == 2) ? -c : s;
  z.im = (quad == 0) ? s : (quad == 1) ? c : (quad == 2) ? -s : -c;
  return z;
}

// Index of the baseline that owns bin k: largest b with koff[b] <= k.  The
// wave's first active lane is searched for by bisection in uniform control
// flow (scalar loads, no dependent vector loads); every lane then steps from
// there to its own baseline, which for the consecutive bins of a wave is
// usually no step at all.  The result stays in [0, n_bl - 1] whatever koff
// holds.
__device__ __forceinline__ int find_baseline(const int64_t* __restrict__ koff, int n_bl, int64_t k) {
  const int64_t k0 = static_cast<int64_t>(
      (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(k >> 32)))) << 32) |
      static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(k & 0xffffffff))));
  int lo = 0, hi = n_bl;  // koff[lo] <= k0 < koff[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (koff[mid] <= k0) lo = mid; else hi = mid;
  }
  int b = lo;
  while (b + 1 < n_bl && koff[b + 1] <= k) ++b;
  while (b > 0 && koff[b] > k) --b;
  return b;
}

// Where bin k lives: baseline, sample and channel ranges, time-bin row.
struct BinRef {
  int b;
  int t0, t1;
  int c0, c1;
  int64_t tb;
};

__device__ __forceinline__ BinRef locate_bin(const int64_t* __restrict__ koff,
                                             const int64_t* __restrict__ tboff,
                                             const int32_t* __restrict__ bl_bin, int n_bl,
                                             int n_t, int n_ch, int64_t k) {
  BinRef r;
  r.b = find_baseline(koff, n_bl, k);
  const int nt = bl_bin[2 * r.b], nc = bl_bin[2 * r.b + 1];
  const int n_fb = (n_ch + nc - 1) / nc;
  const int64_t local = k - koff[r.b];
  // 32-bit division where the bin's index within its baseline allows
  const int T = local <= 0x7fffffff ? static_cast<int>(local) / n_fb : static_cast<int>(local / n_fb);
  const int F = static_cast<int>(local - static_cast<int64_t>(T) * n_fb);
  r.t0 = T * nt;
  r.t1 = min(n_t, r.t0 + nt);
  r.c0 = F * nc;
  r.c1 = min(n_ch, r.c0 + nc);
  r.tb = tboff[r.b] + T;
  return r;
}

// Mean channel frequency of a bin (its centre frequency), FP64.
__device__ __forceinline__ double bin_freq(const double* __restrict__ freq, int c0, int c1) {
  double s = 0.0;
  for (int c = c0; c < c1; ++c) s += freq[c];
  return s / static_cast<double>(c1 - c0);
}

// Pack helpers for the split forms: two floats -> two round-to-nearest
// 16-bit values in one register (one hardware conversion each pair).
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{a, b}, bf16x2_t));
}
// the two halves of a packed bf16 pair, widened back to float (exact)
__device__ __forceinline__ float bf16_lo_to_f32(uint32_t p) { return __builtin_bit_cast(float, p << 16); }
__device__ __forceinline__ float bf16_hi_to_f32(uint32_t p) { return __builtin_bit_cast(float, p & 0xffff0000u); }

__device__ __forceinline__ uint32_t pack_f16x2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{a, b}, f16x2_t));
}
__device__ __forceinline__ float f16_lo_to_f32(uint32_t p) {
  return static_cast<float>(__builtin_bit_cast(f16x2_t, p)[0]);
}
__device__ __forceinline__ float f16_hi_to_f32(uint32_t p) {
  return static_cast<float>(__builtin_bit_cast(f16x2_t, p)[1]);
}
// The lo halves of a split-FP16 pair, v - hi (exact in FP32), written as
// fma(hi, -1, v) with the -1 held in a scalar register so that the compiler
// keeps the multiply-add: with a half-precision source that is one
// mixed-precision instruction per value instead of a conversion and a
// subtraction.  Same values as the plain difference.
__device__ __forceinline__ uint32_t f16_lo_pair(uint32_t hi, float v0, float v1) {
  float m1 = -1.0f;
  asm("" : "+s"(m1));
  return pack_f16x2(__builtin_fmaf(f16_lo_to_f32(hi), m1, v0), __builtin_fmaf(f16_hi_to_f32(hi), m1, v1));
}

}  // namespace psf
