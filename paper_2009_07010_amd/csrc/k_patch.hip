// K-b + K-c/K-e + K-f: phase-factor generation, matrix-core patch
// contraction and the fixed-order split-K finalise.
//
// The patch P_ij = 2 Re sum_k c_k a_ki b_kj, with c_k = W_k D_k,
// a_ki = exp(2 pi i u'_k x_i) and b_kj = exp(2 pi i v'_k y_j), is a real
// matrix product over an inner dimension of 2K:
//   A[k'][i] = (Re(c a), -Im(c a)) = conj(c_k a_ki),  B[k'][j] = (Re b, Im b)
//   P = 2 A^T B.
// The inner dimension runs over visibilities (millions), the output is a
// small patch, so each workgroup owns one output tile and one contiguous
// k-slice, keeps the tile in matrix-core accumulators, and writes a partial
// tile; K-f adds the partials in slice order (deterministic).
//
// Phase factors never touch HBM: for every chunk of KC visibilities the
// workgroup writes A and B columns for its tile into LDS in the exact
// operand layout of the MFMA instruction.  Each 16-pixel run along l (or m)
// is seeded by one FP64-reduced exp(2 pi i u' x) and advanced by the FP64-
// reduced step exp(2 pi i u' dl) in FP32 complex arithmetic.
//
// Split forms: every operand value v is stored as hi = round16(v) and
// lo = round16(v - hi); the product uses hi*hi + hi*lo + lo*hi (three MFMAs)
// with FP32 accumulation.
#include "psf_device.hpp"
#include "psf_kernels.hpp"

namespace psf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// One LDS operand row: 32 16-bit values (16 visibilities x re/im) or 16
// floats (8 visibilities x re/im), 64 bytes, padded to 80 so that 8
// consecutive rows read with 16-byte loads touch 32 distinct banks.
constexpr int kRowBytes = 80;

__device__ __forceinline__ int even_split(int n, int parts, int p) {
  return static_cast<int>((static_cast<int64_t>(n) * p) / parts);
}

template <int PREC>
__device__ __forceinline__ void store_operand(uint8_t* __restrict__ hi_plane, uint8_t* __restrict__ lo_plane,
                                              int sub_bytes, int kl, int row, cf32 z) {
  if constexpr (PREC == kFP32) {
    // group of 8 visibilities; lane group g of the 16x16x4 instruction takes
    // k' = g of each of its 4 k-steps: (re v0, im v0, re v1, im v1)
    const int g = kl >> 3, kv = kl & 7;
    const int step = kv >> 1, gg = (kv & 1) * 2;
    uint8_t* p = hi_plane + g * sub_bytes + row * kRowBytes + gg * 16 + step * 4;
    *reinterpret_cast<float*>(p) = z.re;
    *reinterpret_cast<float*>(p + 16) = z.im;
  } else {
    // k-step of 16 visibilities; lane group g of the 16x16x32 instruction
    // takes k' = 8g..8g+7 = visibilities 4g..4g+3 as (re, im) pairs
    const int s = kl >> 4, kk = kl & 15;
    const int off = s * sub_bytes + row * kRowBytes + kk * 4;
    uint32_t hi, lo = 0;
    if constexpr (PREC == kSplitFP16) {
      hi = pack_f16x2(z.re, z.im);
      lo = pack_f16x2(z.re - f16_lo_to_f32(hi), z.im - f16_hi_to_f32(hi));
    } else {
      hi = pack_bf16x2(z.re, z.im);
      if constexpr (PREC == kSplitBF16) lo = pack_bf16x2(z.re - bf16_lo_to_f32(hi), z.im - bf16_hi_to_f32(hi));
    }
    *reinterpret_cast<uint32_t*>(hi_plane + off) = hi;
    if constexpr (PREC != kPlainBF16) *reinterpret_cast<uint32_t*>(lo_plane + off) = lo;
  }
}

template <int PREC>
__device__ __forceinline__ f32x4 mfma16(const uint8_t* a, const uint8_t* b, f32x4 acc) {
  if constexpr (PREC == kSplitFP16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(*reinterpret_cast<const f16x8*>(a),
                                                  *reinterpret_cast<const f16x8*>(b), acc, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(a),
                                                   *reinterpret_cast<const bf16x8*>(b), acc, 0, 0, 0);
  }
}

template <int PREC, int WM, int WN, int BM, int BN, int KC>
__global__ __launch_bounds__(WM * WN * 64) void k_patch(PatchArgs a) {
  constexpr int NT = WM * WN * 64;
  constexpr int TIM = WM * BM * 16;
  constexpr int TJM = WN * BN * 16;
  constexpr bool kF32 = PREC == kFP32;
  constexpr bool kTwoPlanes = PREC == kSplitBF16 || PREC == kSplitFP16;
  constexpr int NSUB = kF32 ? KC / 8 : KC / 16;
  constexpr int SUBA = TIM * kRowBytes;
  constexpr int SUBB = TJM * kRowBytes;
  constexpr int NPL = kTwoPlanes ? 2 : 1;
  static_assert(KC % 16 == 0, "chunk must hold whole k-steps");
  __shared__ __attribute__((aligned(16))) uint8_t smem[NPL * NSUB * (SUBA + SUBB)];
  uint8_t* const A_hi = smem;
  uint8_t* const A_lo = smem + NSUB * SUBA;
  uint8_t* const B_hi = smem + NPL * NSUB * SUBA;
  uint8_t* const B_lo = B_hi + NSUB * SUBB;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int ti = blockIdx.x / a.tiles_j, tj = blockIdx.x - ti * a.tiles_j;
  const int split = blockIdx.y;
  const int bi0 = even_split(a.nbi, a.tiles_i, ti), nbi_t = even_split(a.nbi, a.tiles_i, ti + 1) - bi0;
  const int bj0 = even_split(a.nbj, a.tiles_j, tj), nbj_t = even_split(a.nbj, a.tiles_j, tj + 1) - bj0;
  const int wm = wave / WN, wn = wave - (wave / WN) * WN;
  const int wi0 = even_split(nbi_t, WM, wm), nwi = even_split(nbi_t, WM, wm + 1) - wi0;
  const int wj0 = even_split(nbj_t, WN, wn), nwj = even_split(nbj_t, WN, wn + 1) - wj0;

  const int64_t kb = static_cast<int64_t>(split) * a.k_per_split;
  const int64_t ke = min(a.K, kb + a.k_per_split);

  f32x4 acc[BM][BN];
#pragma unroll
  for (int r = 0; r < BM; ++r)
#pragma unroll
    for (int c = 0; c < BN; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int ntask = KC * (nbi_t + nbj_t);
  for (int64_t kc = kb; kc < ke; kc += KC) {
    // ---- K-b: phase factors of this chunk into LDS
    for (int t = tid; t < ntask; t += NT) {
      const int kl = t % KC, sg = t / KC;
      const bool isA = sg < nbi_t;
      const int seg = isA ? sg : sg - nbi_t;
      const int64_t kg = kc + kl;
      double f = 0.0;
      cf32 cc = {0.f, 0.f};
      if (kg < ke) {
        const double2 uv = a.uvp[kg];
        f = isA ? uv.x : uv.y;
        const float2 c = a.c[kg];
        cc = {c.x, c.y};
      }
      const int g0 = 16 * ((isA ? bi0 : bj0) + seg);
      const double pos0 = isA ? (a.l_first + g0 * a.dl) - a.l0 : (a.m_first + g0 * a.dm) - a.m0;
      cf32 z = expi_turns(f * pos0);
      cf32 zs = expi_turns(f * (isA ? a.dl : a.dm));
      if (isA) {
        z = conj(cmul(cc, z));
        zs = conj(zs);
      }
      uint8_t* hi = isA ? A_hi : B_hi;
      uint8_t* lo = isA ? A_lo : B_lo;
      const int sub = isA ? SUBA : SUBB;
#pragma unroll 4
      for (int q = 0; q < 16; ++q) {
        store_operand<PREC>(hi, lo, sub, kl, 16 * seg + q, z);
        z = cmul(z, zs);
      }
    }
    __syncthreads();

    // ---- K-c / K-e: matrix-core products over the chunk
#pragma unroll
    for (int s = 0; s < NSUB; ++s) {
      if constexpr (kF32) {
        f32x4 av[BM], bv[BN];
#pragma unroll
        for (int r = 0; r < BM; ++r)
          if (r < nwi)
            av[r] = *reinterpret_cast<const f32x4*>(A_hi + s * SUBA + (16 * (wi0 + r) + lr) * kRowBytes + lg * 16);
#pragma unroll
        for (int c = 0; c < BN; ++c)
          if (c < nwj)
            bv[c] = *reinterpret_cast<const f32x4*>(B_hi + s * SUBB + (16 * (wj0 + c) + lr) * kRowBytes + lg * 16);
#pragma unroll
        for (int r = 0; r < BM; ++r)
#pragma unroll
          for (int c = 0; c < BN; ++c)
            if (r < nwi && c < nwj) {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r][e], bv[c][e], acc[r][c], 0, 0, 0);
            }
      } else {
        const uint8_t* pa[BM];
        const uint8_t* pb[BN];
#pragma unroll
        for (int r = 0; r < BM; ++r) pa[r] = A_hi + s * SUBA + (16 * (wi0 + r) + lr) * kRowBytes + lg * 16;
#pragma unroll
        for (int c = 0; c < BN; ++c) pb[c] = B_hi + s * SUBB + (16 * (wj0 + c) + lr) * kRowBytes + lg * 16;
#pragma unroll
        for (int r = 0; r < BM; ++r)
#pragma unroll
          for (int c = 0; c < BN; ++c)
            if (r < nwi && c < nwj) {
              acc[r][c] = mfma16<PREC>(pa[r], pb[c], acc[r][c]);
              if constexpr (kTwoPlanes) {
                acc[r][c] = mfma16<PREC>(pa[r], pb[c] + NSUB * SUBB, acc[r][c]);
                acc[r][c] = mfma16<PREC>(pa[r] + NSUB * SUBA, pb[c], acc[r][c]);
              }
            }
      }
    }
    __syncthreads();
  }

  // ---- partial tile of this k-slice
  const int width = 16 * a.nbj;
  float* out = a.partial + static_cast<size_t>(split) * (16 * a.nbi) * width;
#pragma unroll
  for (int r = 0; r < BM; ++r)
#pragma unroll
    for (int c = 0; c < BN; ++c)
      if (r < nwi && c < nwj) {
        const int col = 16 * (bj0 + wj0 + c) + lr;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = 16 * (bi0 + wi0 + r) + 4 * lg + e;
          out[static_cast<size_t>(row) * width + col] = acc[r][c][e];
        }
      }
}

// K-f: P = 2 * sum over k-slices, in slice order.
__global__ __launch_bounds__(256) void k_finalize(const float* __restrict__ partial, int n_split, int nbi,
                                                  int nbj, int nl, int nm, float* __restrict__ P) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(nl) * nm) return;
  const int i = static_cast<int>(idx / nm), j = static_cast<int>(idx - static_cast<int64_t>(i) * nm);
  const size_t plane = static_cast<size_t>(16 * nbi) * (16 * nbj);
  const size_t off = static_cast<size_t>(i) * (16 * nbj) + j;
  float s = 0.f;
  for (int p = 0; p < n_split; ++p) s += partial[p * plane + off];
  P[idx] = 2.0f * s;
}

constexpr int kWM = 2, kWN = 2, kBM = 5, kBN = 5, kKC = 32;

PatchShape patch_shape(int /*prec*/) { return PatchShape{kWM, kWN, kBM, kBN, kKC}; }

hipError_t launch_patch(int prec, const PatchArgs& a, hipStream_t stream) {
  const dim3 grid(static_cast<unsigned>(a.tiles_i * a.tiles_j), static_cast<unsigned>(a.n_split));
  const dim3 block(kWM * kWN * 64);
  switch (prec) {
    case kFP32:
      hipLaunchKernelGGL((k_patch<kFP32, kWM, kWN, kBM, kBN, kKC>), grid, block, 0, stream, a);
      break;
    case kSplitBF16:
      hipLaunchKernelGGL((k_patch<kSplitBF16, kWM, kWN, kBM, kBN, kKC>), grid, block, 0, stream, a);
      break;
    case kSplitFP16:
      hipLaunchKernelGGL((k_patch<kSplitFP16, kWM, kWN, kBM, kBN, kKC>), grid, block, 0, stream, a);
      break;
    case kPlainBF16:
      hipLaunchKernelGGL((k_patch<kPlainBF16, kWM, kWN, kBM, kBN, kKC>), grid, block, 0, stream, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const float* partial, int n_split, int nbi, int nbj, int nl, int nm, float* P,
                           hipStream_t stream) {
  const int64_t n = static_cast<int64_t>(nl) * nm;
  const int threads = 256;
  hipLaunchKernelGGL(k_finalize, dim3(static_cast<unsigned>((n + threads - 1) / threads)), dim3(threads), 0,
                     stream, partial, n_split, nbi, nbj, nl, nm, P);
  return hipGetLastError();
}

}  // namespace psf
