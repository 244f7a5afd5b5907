// Reverse-mode adjoint of the patch for patches of up to 288 columns (and
// rows within 16 ranges that fit in LDS) in the FP32, split-BF16 and
// split-FP16 forms.  The derivatives are those of the
// five-patch form in psf_backward.hip (derivation in k_decorr.hip),
// regrouped per visibility:
//   dL/dl0 = 2 Re sum_k [e0_k H_k + e2_k Hx_k + e3_k Hy_k]
//   dL/dm0 = 2 Re sum_k [e1_k H_k + e3_k Hx_k + e4_k Hy_k]
// with H_k = sum_ij G_ij a_ki b_kj, Hx_k = sum_ij x_i G_ij a_ki b_kj and
// Hy_k = sum_ij y_j G_ij a_ki b_kj (G = dL/dP, a and b the phase factors of
// the forward patch).  Per visibility this needs the column T = G b_k and
// Ty = G (y o b_k) (matrix-core products, G resident in LDS) and three dot
// products with a_k (vector registers): two products of the patch's size per
// visibility instead of five derivative patches.
//
// Layout: one workgroup of four waves (one per SIMD) per (k-slice, range of
// row blocks whose G fragments fit in LDS): H is a sum over rows, so the row
// ranges' shares of the gradient add.  G's rows of the range, scaled by a power of two (FP16
// range) and split hi + lo, sit in LDS as 16x32 operand fragments
// [row block][k-step][hi/lo][lane][8 values].  A wave takes
// 16 visibilities at a time; lane l owns visibility l mod 16 and generates
// the 8 consecutive columns 32 s + 8 (l / 16) .. + 7 of its b for k-step s
// (the operand layout of the 16x16x32 instructions), and after the products
// holds T at rows 16 r + 4 (l / 16) + e, e = 0..3, of the same visibility.
//
// Folded columns (split forms, odd patch widths nm = 2c + 1).  With
// y_j = delta + t_j dm, t_j = j - c, and b_kj = e_k z_k(t_j), e_k =
// exp(2 pi i v'_k delta), z(t) = C(t) + i S(t) = exp(2 pi i v' t dm):
//   sum_j G_ij b_kj     = e_k [sum_t Ge_it C(t) + i sum_t Go_it S(t)]
//   sum_j G_ij t_j dm b_kj = e_k [sum_t Go_it t dm C(t) + i sum_t Ge_it t dm S(t)]
// with Ge_it = G_i,c+t + G_i,c-t (Ge_i0 = G_ic) and Go_it = G_i,c+t - G_i,c-t,
// t >= 0.  G is folded once into Ge (c + 1 columns) and Go (c columns) in
// LDS, and each visibility needs four real products over half the columns
// (Ge C, Ge t S, Go S, Go t C) instead of four over all of them: half the
// matrix-core work.  Then T = e_k (Ge C + i Go S) and
// G (y o b_k) = delta T + e_k (Go t C + i Ge t S).
#include <algorithm>
#include <cmath>

#include "psf_device.hpp"
#include "psf_host.hpp"

namespace psf {

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) uint8_t lds_b;
typedef __attribute__((address_space(3))) v4u lds_v4u;

constexpr int kAdjThreads = 256;  // four waves, one per SIMD
constexpr int kAdjMaxRB = 9;      // row blocks of 16 per workgroup
constexpr int kAdjMaxKS = 9;      // k-steps of 32 columns: nm <= 288
constexpr int kAdjMaxFrags = 72;  // G fragment pairs in LDS (144 KiB)
constexpr int kAdjMaxRanges = 16; // row ranges per patch
constexpr int kAdjSlices = 512;   // k-slices per source
constexpr int kFragBytes = 1024;  // one 16x32 16-bit operand fragment

struct AdjArgs {
  const BinRec* rec;
  const float2* coef;  // e0..e4, vector q at coef + q K
  const float* G;      // [nl][nm]
  double* partial;     // [ranges][slices][2]
  int64_t K, slice;
  int rb_per_range;    // row blocks per range (the last range may have fewer)
  double l_first, m_first, dl, dm, l0, m0;
  const double* dir;   // if not null: the values above from device memory (psf_src layout)
  int nl, nm, nks;
  int nke;             // folded columns: k-steps of Ge (those of Go follow, nks - nke)
};

template <int PREC>
__device__ __forceinline__ v4f mma(const v4u& a, const v4u& b, v4f c) {
  if constexpr (PREC == kSplitFP16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a), __builtin_bit_cast(v8h, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0,
                                                   0);
}

// Two values into packed 16-bit hi and lo parts (lo = v - hi, exact in FP32).
template <int PREC>
__device__ __forceinline__ void split2(float p, float q, uint32_t& hi, uint32_t& lo) {
  if constexpr (PREC == kSplitFP16) {
    hi = pack_f16x2(p, q);
    lo = f16_lo_pair(hi, p, q);
  } else {
    hi = pack_bf16x2(p, q);
    lo = pack_bf16x2(p - bf16_lo_to_f32(hi), q - bf16_hi_to_f32(hi));
  }
}

__device__ __forceinline__ int frag_off(int rb, int ks, int nks, int part) {
  return ((rb * nks + ks) * 2 + part) * kFragBytes;
}

constexpr int frag_capacity(int nrb) { return nrb * kAdjMaxKS < kAdjMaxFrags ? nrb * kAdjMaxKS : kAdjMaxFrags; }

template <int PREC, int NRB, bool FOLD>
__global__ __launch_bounds__(kAdjThreads) void k_adjoint(AdjArgs a) {
  static_assert(!FOLD || PREC != kFP32, "folded columns are built for the split forms");
  // NRB * nks <= frag_capacity(NRB) (checked on the host)
  __shared__ __attribute__((aligned(16))) uint8_t lds_raw[frag_capacity(NRB) * 2 * kFragBytes];
  __shared__ float s_red[kAdjThreads / 64];
  __shared__ double s_g[2][kAdjThreads / 64];
  lds_b* lds = (lds_b*)lds_raw;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rb0 = blockIdx.y * a.rb_per_range;  // first row block of this range
  const int nrb = min(NRB, (a.nl + 15) / 16 - rb0);

  // G's scale: a power of two with max |G| scale < 2^14 (FP16); 1 for BF16.
  float g_scale = 1.0f;
  if constexpr (PREC == kSplitFP16) {
    float mx = 0.0f;
    for (int p = threadIdx.x; p < a.nl * a.nm; p += kAdjThreads) mx = fmaxf(mx, fabsf(a.G[p]));
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (lane == 0) s_red[wave] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3]));
    if (mx > 0.0f) {
      int e;
      frexpf(mx, &e);  // mx < 2^e
      g_scale = ldexpf(1.0f, 14 - e);
    }
  }
  // G into LDS as operand fragments; rows >= nl and columns >= nm are 0.
  // FP32: per 32 columns eight 16x4 fragments of 64 floats (lane l: row
  // l mod 16, column 4 k4 + l / 16), in the same 2 KiB as a split pair.
  if constexpr (PREC == kFP32) {
    const int n_f32 = NRB * a.nks * 8 * 64;
    for (int it = threadIdx.x; it < n_f32; it += kAdjThreads) {
      const int l = it & 63, f = it >> 6;
      const int k4 = f & 7, f2 = f >> 3;
      const int rb = f2 / a.nks, ks = f2 - rb * a.nks;
      const int i = 16 * (rb0 + rb) + (l & 15), j = 32 * ks + 4 * k4 + (l >> 4);
      const float v = (i < a.nl && j < a.nm) ? a.G[static_cast<int64_t>(i) * a.nm + j] : 0.0f;
      *reinterpret_cast<__attribute__((address_space(3))) float*>(lds + frag_off(rb, ks, a.nks, 0) + k4 * 256 +
                                                                    l * 4) = v;
    }
  }
  const int n_items = PREC == kFP32 ? 0 : NRB * a.nks * 64;
  for (int it = threadIdx.x; it < n_items; it += kAdjThreads) {
    const int l = it & 63, f = it >> 6;
    const int rb = f / a.nks, ks = f - rb * a.nks;
    const int i = 16 * (rb0 + rb) + (l & 15), j0 = 32 * ks + 8 * (l >> 4);
    float v[8];
    if constexpr (FOLD) {
      // Ge k-steps: t = 32 ks + 8 (l / 16) + u; Go k-steps: that of ks - nke, plus 1
      const int c = (a.nm - 1) / 2;
      const bool even = ks < a.nke;
      const int t0 = (even ? 32 * ks : 32 * (ks - a.nke) + 1) + 8 * (l >> 4);
      const float* row = a.G + static_cast<int64_t>(i) * a.nm;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + u;
        float g = 0.0f;
        if (i < a.nl && t <= c) {
          const float hi = row[c + t], lo = row[c - t];
          g = even ? (t == 0 ? hi : hi + lo) : hi - lo;
        }
        v[u] = g * g_scale;
      }
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int j = j0 + t;
        v[t] = (i < a.nl && j < a.nm) ? a.G[static_cast<int64_t>(i) * a.nm + j] * g_scale : 0.0f;
      }
    }
    v4u hi, lo;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      uint32_t h, w;
      split2<PREC>(v[2 * t], v[2 * t + 1], h, w);
      hi[t] = h;
      lo[t] = w;
    }
    *reinterpret_cast<lds_v4u*>(lds + frag_off(rb, ks, a.nks, 0) + l * 16) = hi;
    *reinterpret_cast<lds_v4u*>(lds + frag_off(rb, ks, a.nks, 1) + l * 16) = lo;
  }
  __syncthreads();

  const int n = lane & 15, jg = lane >> 4;
  (void)nrb;
  const int64_t kb = static_cast<int64_t>(blockIdx.x) * a.slice;
  const int64_t ke = min(a.K, kb + a.slice);
  double l0 = a.l0, m0 = a.m0, l_first = a.l_first, m_first = a.m_first, dl = a.dl, dm = a.dm;
  if (a.dir != nullptr) {
    l0 = a.dir[0];
    m0 = a.dir[1];
    l_first = a.dir[2];
    m_first = a.dir[3];
    dl = a.dir[4];
    dm = a.dir[5];
  }
  // y offsets of the grid: |y_j| < 2^e for all j, so y 2^-e lies in (-1, 1)
  double y_scale = 1.0;
  {
    const double ymax = fmax(fabs(m_first - m0), fabs(m_first + (a.nm - 1) * dm - m0));
    int e = 0;
    if (ymax > 0.0) frexp(ymax, &e);
    y_scale = ldexp(1.0, -e);
  }
  // folded columns: offsets t dm from the centre column c, |t dm| t_scale < 1,
  // and the centre column's offset from the source
  const int cc = (a.nm - 1) / 2;
  double t_scale = 1.0;
  {
    const double tmax = fabs(cc * dm);
    int e = 0;
    if (tmax > 0.0) frexp(tmax, &e);
    t_scale = ldexp(1.0, -e);
  }
  const double delta_m = (m_first + cc * dm) - m0;
  const float inv_t = static_cast<float>(1.0 / t_scale), tds = static_cast<float>(dm * t_scale);
  (void)inv_t;
  (void)tds;
  const float inv_y = static_cast<float>(1.0 / y_scale);
  // first column of the lane: 8 jg (16-bit operands), jg (FP32 operands)
  const double y_lane = (m_first + (PREC == kFP32 ? jg : 8 * jg) * dm) - m0;
  const double x_lane = (l_first + (16 * rb0 + 4 * jg) * dl) - l0;  // row 16 rb0 + 4 jg
  const float ys0 = static_cast<float>(y_lane * y_scale), ystep = static_cast<float>(dm * y_scale);
  const float xs0 = static_cast<float>(x_lane), xstep = static_cast<float>(dl);
  double gl = 0.0, gm = 0.0;
  for (int64_t k0 = kb + 16 * wave; k0 < ke; k0 += 16 * (kAdjThreads / 64)) {
    const int64_t kk = k0 + n;
    const bool ok = kk < ke;
    const BinRec* r = a.rec + (ok ? kk : ke - 1);
    const double up = r->up, vp = r->vp;
    cf32 zb = expi_turns(vp * y_lane);
    v4f acc[NRB][4];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[rb][q] = v4f{0.f, 0.f, 0.f, 0.f};
    if constexpr (PREC == kFP32) {
      // one column per lane and 16x16x4 step: columns jg, jg + 4, ...
      const cf32 s4 = expi_turns(vp * (4.0 * dm));
      for (int ks = 0; ks < a.nks; ++ks) {
#pragma unroll
        for (int k4 = 0; k4 < 8; ++k4) {
          const float y = ys0 + static_cast<float>(32 * ks + 4 * k4) * ystep;
          const cf32 b = zb;
          zb = cmul(zb, s4);
          const float yr = y * b.re, yi = y * b.im;
#pragma unroll
          for (int rb = 0; rb < NRB; ++rb) {
            const float g = *reinterpret_cast<const __attribute__((address_space(3))) float*>(
                lds + frag_off(rb, ks, a.nks, 0) + k4 * 256 + lane * 4);
            acc[rb][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(g, b.re, acc[rb][0], 0, 0, 0);
            acc[rb][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(g, b.im, acc[rb][1], 0, 0, 0);
            acc[rb][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(g, yr, acc[rb][2], 0, 0, 0);
            acc[rb][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(g, yi, acc[rb][3], 0, 0, 0);
          }
        }
      }
    }
    // Along a lane's 8 consecutive columns the factors follow the real
    // three-term recurrence z+ = 2 cos(t) z - z- of the column step e^{it}
    // (two fused multiply-adds per column; over 8 columns an element stays
    // within 3e-6, under the split representation's rounding); the jump to
    // the next k-step's first column, and its predecessor, are complex
    // products from the current value, so the error carries from k-step to
    // k-step: over a row of up to 9 k-steps (288 columns) at most about
    // 3e-5 of an element in the worst case (the smallest column steps),
    // incoherent across visibilities (the gradients of 257-column patches
    // with column steps of 1e-5 to 1e-4 rad stay within 3e-7).
    const cf32 s1 = expi_turns(vp * dm), s25 = expi_turns(vp * (25.0 * dm));
    const cf32 s24 = cmul(s25, conj(s1));
    const float tc = 2.0f * s1.re;
    cf32 zp = cmul(zb, conj(s1));  // the column before zb
    if constexpr (FOLD) {
      // Ge k-steps (t = 32 ks + 8 jg + u: C into product 0, t dm S into 1),
      // then Go k-steps (t = 32 (ks - nke) + 8 jg + u + 1: S into 2, t dm C
      // into 3); each half seeded once at its first column (FP64-reduced)
      for (int half = 0; half < 2; ++half) {
        const int ks0 = half == 0 ? 0 : a.nke, ks1 = half == 0 ? a.nke : a.nks;
        const int tl = 8 * jg + half;  // the lane's first t of the half
        zb = expi_turns(vp * (tl * dm));
        zp = cmul(zb, conj(s1));
        for (int ks = ks0; ks < ks1; ++ks) {
          v4u bh[2], bl[2];
          const int tk = tl + 32 * (ks - ks0);
#pragma unroll
          for (int u = 0; u < 8; u += 2) {
            const cf32 z0 = zb;
            const cf32 z1 = {__builtin_fmaf(tc, z0.re, -zp.re), __builtin_fmaf(tc, z0.im, -zp.im)};
            zp = z1;
            zb = z1;
            if (u < 6) zb = {__builtin_fmaf(tc, z1.re, -z0.re), __builtin_fmaf(tc, z1.im, -z0.im)};
            const float t0 = static_cast<float>(tk + u) * tds, t1 = t0 + tds;
            uint32_t h, w;
            split2<PREC>(half == 0 ? z0.re : z0.im, half == 0 ? z1.re : z1.im, h, w);
            bh[0][u / 2] = h;
            bl[0][u / 2] = w;
            split2<PREC>(t0 * (half == 0 ? z0.im : z0.re), t1 * (half == 0 ? z1.im : z1.re), h, w);
            bh[1][u / 2] = h;
            bl[1][u / 2] = w;
          }
          zp = cmul(zb, s24);
          zb = cmul(zb, s25);
#pragma unroll
          for (int rb = 0; rb < NRB; ++rb) {
            const v4u gh = *reinterpret_cast<const lds_v4u*>(lds + frag_off(rb, ks, a.nks, 0) + lane * 16);
            const v4u gw = *reinterpret_cast<const lds_v4u*>(lds + frag_off(rb, ks, a.nks, 1) + lane * 16);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              v4f& ac = acc[rb][2 * half + q];
              ac = mma<PREC>(gh, bh[q], ac);
              ac = mma<PREC>(gh, bl[q], ac);
              ac = mma<PREC>(gw, bh[q], ac);
            }
          }
        }
      }
    }
    for (int ks = 0; ks < (PREC == kFP32 || FOLD ? 0 : a.nks); ++ks) {
      // b and y b at columns 32 ks + 8 jg + t, t = 0..7: re, im, y re, y im
      v4u bh[4], bl[4];
#pragma unroll
      for (int t = 0; t < 8; t += 2) {
        const cf32 z0 = zb;
        const cf32 z1 = {__builtin_fmaf(tc, z0.re, -zp.re), __builtin_fmaf(tc, z0.im, -zp.im)};
        zp = z1;
        zb = z1;
        if (t < 6) zb = {__builtin_fmaf(tc, z1.re, -z0.re), __builtin_fmaf(tc, z1.im, -z0.im)};
        const float y0 = ys0 + static_cast<float>(32 * ks + t) * ystep, y1 = y0 + ystep;
        uint32_t h, w;
        split2<PREC>(z0.re, z1.re, h, w);
        bh[0][t / 2] = h;
        bl[0][t / 2] = w;
        split2<PREC>(z0.im, z1.im, h, w);
        bh[1][t / 2] = h;
        bl[1][t / 2] = w;
        split2<PREC>(y0 * z0.re, y1 * z1.re, h, w);
        bh[2][t / 2] = h;
        bl[2][t / 2] = w;
        split2<PREC>(y0 * z0.im, y1 * z1.im, h, w);
        bh[3][t / 2] = h;
        bl[3][t / 2] = w;
      }
      zp = cmul(zb, s24);  // column 32 (ks + 1) + 8 jg - 1
      zb = cmul(zb, s25);  // column 32 ks + 8 jg + 7 -> 32 (ks + 1) + 8 jg
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) {
        const v4u gh = *reinterpret_cast<const lds_v4u*>(lds + frag_off(rb, ks, a.nks, 0) + lane * 16);
        const v4u gw = *reinterpret_cast<const lds_v4u*>(lds + frag_off(rb, ks, a.nks, 1) + lane * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[rb][q] = mma<PREC>(gh, bh[q], acc[rb][q]);
          acc[rb][q] = mma<PREC>(gh, bl[q], acc[rb][q]);
          acc[rb][q] = mma<PREC>(gw, bh[q], acc[rb][q]);
        }
      }
    }
    // H, Hx, Hy over this lane's rows 16 rb + 4 jg + e
    cf32 za = expi_turns(up * x_lane);
    const cf32 t1 = expi_turns(up * dl), t13 = expi_turns(up * (13.0 * dl));
    float h1r = 0.f, h1i = 0.f, hxr = 0.f, hxi = 0.f, hyr = 0.f, hyi = 0.f;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float x = xs0 + static_cast<float>(16 * rb + e) * xstep;
        // T (re, im) and G (y o b) (re, im); folded: Ge C, Go S and Go t C, Ge t S
        const float tr = acc[rb][0][e], ti = acc[rb][FOLD ? 2 : 1][e];
        const float ar = za.re * tr - za.im * ti, ai = za.re * ti + za.im * tr;
        h1r += ar;
        h1i += ai;
        hxr += x * ar;
        hxi += x * ai;
        const float ur = acc[rb][FOLD ? 3 : 2][e], ui = acc[rb][FOLD ? 1 : 3][e];
        hyr += za.re * ur - za.im * ui;
        hyi += za.re * ui + za.im * ur;
        za = cmul(za, e < 3 ? t1 : t13);
      }
    }
    // the four lane groups of a visibility hold disjoint rows
    for (int o = 16; o <= 32; o <<= 1) {
      h1r += __shfl_xor(h1r, o);
      h1i += __shfl_xor(h1i, o);
      hxr += __shfl_xor(hxr, o);
      hxi += __shfl_xor(hxi, o);
      hyr += __shfl_xor(hyr, o);
      hyi += __shfl_xor(hyi, o);
    }
    if (jg == 0 && ok) {
      if constexpr (FOLD) {
        // the centre column's factor e_k = exp(2 pi i v' delta) on every sum,
        // and G (y o b) = delta T + e_k G (t dm b) (the latter scaled by t_scale)
        const cf32 ek = expi_turns(vp * delta_m);
        const cf32 H = cmul(ek, cf32{h1r, h1i}), Hx = cmul(ek, cf32{hxr, hxi});
        const cf32 Ht = cmul(ek, cf32{hyr * inv_t, hyi * inv_t});
        const float dm_f = static_cast<float>(delta_m);
        h1r = H.re;
        h1i = H.im;
        hxr = Hx.re;
        hxi = Hx.im;
        hyr = __builtin_fmaf(dm_f, H.re, Ht.re);
        hyi = __builtin_fmaf(dm_f, H.im, Ht.im);
      } else {
        hyr *= inv_y;
        hyi *= inv_y;
      }
      const float2 e0 = a.coef[kk], e1 = a.coef[a.K + kk], e2 = a.coef[2 * a.K + kk];
      const float2 e3 = a.coef[3 * a.K + kk], e4 = a.coef[4 * a.K + kk];
      auto re = [](float2 c, float hr, float hi) {
        return static_cast<double>(c.x) * hr - static_cast<double>(c.y) * hi;
      };
      gl += 2.0 * (re(e0, h1r, h1i) + re(e2, hxr, hxi) + re(e3, hyr, hyi));
      gm += 2.0 * (re(e1, h1r, h1i) + re(e3, hxr, hxi) + re(e4, hyr, hyi));
    }
  }
  // fixed-order workgroup sum
  for (int o = 32; o > 0; o >>= 1) {
    gl += __shfl_xor(gl, o);
    gm += __shfl_xor(gm, o);
  }
  if (lane == 0) {
    s_g[0][wave] = gl;
    s_g[1][wave] = gm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sl = 0.0, sm = 0.0;
    for (int w = 0; w < kAdjThreads / 64; ++w) {
      sl += s_g[0][w];
      sm += s_g[1][w];
    }
    const int64_t slot = static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x;
    a.partial[2 * slot] = sl / g_scale;
    a.partial[2 * slot + 1] = sm / g_scale;
  }
}

// grad = (sum of the workgroup partials in order) / kAdjointScale
__global__ __launch_bounds__(256) void k_adjoint_sum(const double* __restrict__ partial, int n,
                                                     double* __restrict__ grad) {
  __shared__ double s[2][256];
  double gl = 0.0, gm = 0.0;
  for (int w = threadIdx.x; w < n; w += 256) {
    gl += partial[2 * w];
    gm += partial[2 * w + 1];
  }
  s[0][threadIdx.x] = gl;
  s[1][threadIdx.x] = gm;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (static_cast<int>(threadIdx.x) < o) {
      s[0][threadIdx.x] += s[0][threadIdx.x + o];
      s[1][threadIdx.x] += s[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    grad[0] = s[0][0] / kAdjointScale;
    grad[1] = s[1][0] / kAdjointScale;
  }
}

template <int PREC, bool FOLD>
hipError_t launch_rb(int nrb, const AdjArgs& a, int n_wg, int n_ranges, hipStream_t st) {
  const dim3 g(n_wg, n_ranges), b(kAdjThreads);
  switch (nrb) {
    case 1: hipLaunchKernelGGL((k_adjoint<PREC, 1, FOLD>), g, b, 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_adjoint<PREC, 2, FOLD>), g, b, 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_adjoint<PREC, 3, FOLD>), g, b, 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_adjoint<PREC, 4, FOLD>), g, b, 0, st, a); break;
    case 5: hipLaunchKernelGGL((k_adjoint<PREC, 5, FOLD>), g, b, 0, st, a); break;
    case 6: hipLaunchKernelGGL((k_adjoint<PREC, 6, FOLD>), g, b, 0, st, a); break;
    case 7: hipLaunchKernelGGL((k_adjoint<PREC, 7, FOLD>), g, b, 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_adjoint<PREC, 8, FOLD>), g, b, 0, st, a); break;
    default: hipLaunchKernelGGL((k_adjoint<PREC, 9, FOLD>), g, b, 0, st, a); break;
  }
  return hipGetLastError();
}

// Row ranges of a patch: each range's G fragments (its row blocks times the
// k-steps) fit in LDS.
struct RowRanges {
  int nks, nke, n_ranges, rb_per_range;
};
// Folded columns for the split forms and odd widths (nm = 2c + 1): Ge has
// c + 1 columns, Go c, each padded to k-steps of 32.
bool fold_columns(int prec, const psf_src& s) { return prec != kFP32 && (s.nm & 1) == 1; }
RowRanges row_ranges(const psf_src& s, bool fold) {
  RowRanges r;
  const int c = (s.nm - 1) / 2;
  r.nke = fold ? (c + 32) / 32 : 0;
  r.nks = fold ? r.nke + (c + 31) / 32 : (s.nm + 31) / 32;
  const int max_rb = std::min(kAdjMaxRB, kAdjMaxFrags / std::max(1, r.nks));
  const int nb = (s.nl + 15) / 16;
  r.n_ranges = (nb + max_rb - 1) / max_rb;
  r.rb_per_range = (nb + r.n_ranges - 1) / r.n_ranges;
  return r;
}

}  // namespace

bool adjoint_reverse_ok(int prec, const psf_obs* o, const psf_src& s) {
  if (!(prec == kSplitBF16 || prec == kSplitFP16 || prec == kFP32) || o->K <= 0) return false;
  const RowRanges r = row_ranges(s, fold_columns(prec, s));
  return r.nks <= kAdjMaxKS && r.n_ranges <= kAdjMaxRanges;
}

size_t adjoint_reverse_partial_bytes() {
  return static_cast<size_t>(kAdjSlices) * kAdjMaxRanges * 2 * sizeof(double);
}

hipError_t launch_adjoint_reverse(const psf_obs* o, const psf_src& s, int prec, const BinRec* rec,
                                  const float2* coef, const float* G, double* partial, double* grad,
                                  hipStream_t st, const double* dir) {
  AdjArgs a;
  a.rec = rec;
  a.coef = coef;
  a.G = G;
  a.partial = partial;
  a.K = o->K;
  // row ranges of equal size, each range's G fragments within LDS
  const bool fold = fold_columns(prec, s);
  const RowRanges rr = row_ranges(s, fold);
  a.nks = rr.nks;
  a.nke = rr.nke;
  a.rb_per_range = rr.rb_per_range;
  const int n_ranges = rr.n_ranges;
  // fewer k-slices when there are several ranges: about kAdjSlices workgroups
  const int slices = std::max(1, kAdjSlices / n_ranges);
  const int64_t per = (o->K + slices - 1) / slices;
  a.slice = std::max<int64_t>(64, (per + 63) / 64 * 64);
  const int n_wg = static_cast<int>(std::min<int64_t>(slices, (o->K + a.slice - 1) / a.slice));
  a.l_first = s.l_first;
  a.m_first = s.m_first;
  a.dl = s.dl;
  a.dm = s.dm;
  a.l0 = s.l0;
  a.m0 = s.m0;
  a.dir = dir;
  a.nl = s.nl;
  a.nm = s.nm;
  const int nrb = a.rb_per_range;
  hipError_t err = prec == kFP32 ? launch_rb<kFP32, false>(nrb, a, n_wg, n_ranges, st)
                   : prec == kSplitFP16
                       ? (fold ? launch_rb<kSplitFP16, true>(nrb, a, n_wg, n_ranges, st)
                               : launch_rb<kSplitFP16, false>(nrb, a, n_wg, n_ranges, st))
                       : (fold ? launch_rb<kSplitBF16, true>(nrb, a, n_wg, n_ranges, st)
                               : launch_rb<kSplitBF16, false>(nrb, a, n_wg, n_ranges, st));
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_adjoint_sum, dim3(1), dim3(256), 0, st, partial, n_wg * n_ranges, grad);
  return hipGetLastError();
}

}  // namespace psf
