// Device-side building blocks shared by the kernels of libpsfdecorr (gfx950).
//
// Phase factors exp(2 pi i theta) with theta in turns: theta is formed in
// FP64 (u' x reaches tens of turns, u l0 thousands), reduced to its
// fractional part in FP64 -- exact, since subtracting the nearest integer
// loses nothing -- and only then converted to FP32 for sin/cos.
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

// Fractional part of theta (turns) in [-1/2, 1/2], computed in FP64.
__device__ __forceinline__ double reduce_turns(double theta) { return theta - rint(theta); }

// exp(2 pi i r) for |r| <= 1/2 turns, FP32.
__device__ __forceinline__ cf32 expi_turns_f32(float r) {
  float s, c;
  sincospif(2.0f * r, &s, &c);
  return {c, s};
}

// exp(2 pi i theta): FP64 argument reduction, FP32 evaluation.
__device__ __forceinline__ cf32 expi_turns(double theta) {
  return expi_turns_f32(static_cast<float>(reduce_turns(theta)));
}

// Index of the baseline that owns bin k: largest b with koff[b] <= k.
__device__ __forceinline__ int find_baseline(const int64_t* __restrict__ koff, int n_bl, int64_t k) {
  int lo = 0, hi = n_bl;  // koff[lo] <= k < koff[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (koff[mid] <= k) lo = mid; else hi = mid;
  }
  return lo;
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
  const int T = static_cast<int>(local / n_fb);
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

// Pack helpers for the split forms: hi = round(x), lo = round(x - hi).
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  __bf16 ha = static_cast<__bf16>(a), hb = static_cast<__bf16>(b);
  uint16_t ua = __builtin_bit_cast(uint16_t, ha), ub = __builtin_bit_cast(uint16_t, hb);
  return static_cast<uint32_t>(ua) | (static_cast<uint32_t>(ub) << 16);
}
__device__ __forceinline__ float bf16_lo_to_f32(uint32_t p) { return __builtin_bit_cast(float, p << 16); }
__device__ __forceinline__ float bf16_hi_to_f32(uint32_t p) { return __builtin_bit_cast(float, p & 0xffff0000u); }

__device__ __forceinline__ uint32_t pack_f16x2(float a, float b) {
  _Float16 ha = static_cast<_Float16>(a), hb = static_cast<_Float16>(b);
  uint16_t ua = __builtin_bit_cast(uint16_t, ha), ub = __builtin_bit_cast(uint16_t, hb);
  return static_cast<uint32_t>(ua) | (static_cast<uint32_t>(ub) << 16);
}
__device__ __forceinline__ float f16_lo_to_f32(uint32_t p) {
  return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(p & 0xffffu)));
}
__device__ __forceinline__ float f16_hi_to_f32(uint32_t p) {
  return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(p >> 16)));
}

}  // namespace psf
