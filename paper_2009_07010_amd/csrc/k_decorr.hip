// K-a: decorrelation factor of every averaged visibility, and the per-bin
// records the patch contraction consumes.
//
// For bin k (baseline b, samples t in [t0,t1), channels c in [c0,c1)) and
// source direction L = (l0, m0, n0 - 1):
//   A_t = uvw_m[b][t] . L          (metres, FP64)
//   A_k = uvw_c_m[tb] . L
//   phi(t, c) = (A_t nu_c - A_k nu_k) / c          (turns, FP64)
//   D_k = mean exp(-2 pi i phi)                    [section 2.3 averaging;
//                                                   section 3.1 factorisation]
// Both products are rounded separately before the difference, so a
// one-sample bin (uvw_c = uvw_m row, nu_k = nu_c) gives phi = 0 exactly and
// D = 1 exactly, as does the phase centre.
//
// Derivatives for the adjoint: d phi/d l0 = du - dw l0/n0, d phi/d m0 =
// dv - dw m0/n0 (du = (u_t nu_c - u_k nu_k)/c etc.), so
// dD/dl0 = mean(-2 pi i dphi/dl0 exp(-2 pi i phi)).
//
// With c_k = W_k D_k, a_ki = exp(2 pi i u'_k x_i), b_kj = exp(2 pi i v'_k
// y_j) and the pixel grid fixed (x_i = l_i - l0, y_j = m_j - m0):
//   dP_ij/dl0 = 2 Re sum_k a_ki b_kj [W_k dD_k/dl0
//               + 2 pi i c_k (du'_k/dl0 x_i + dv'_k/dl0 y_j - u'_k)]
// and likewise for m0 (with -v'_k), where
//   du'/dl0 = -w (1 - m0^2)/n0^3, du'/dm0 = dv'/dl0 = -w l0 m0/n0^3,
//   dv'/dm0 = -w (1 - l0^2)/n0^3.
// So every derivative patch is a sum of patches of the same form as P with
// c_k replaced by one of five coefficient vectors, weighted by 1, x_i or y_j:
//   e0 = W dD/dl0 - 2 pi i c u'    (weight 1, for l0)
//   e1 = W dD/dm0 - 2 pi i c v'    (weight 1, for m0)
//   e2 = 2 pi i c du'/dl0          (weight x_i, for l0)
//   e3 = 2 pi i c dv'/dl0          (weight y_j for l0; weight x_i for m0)
//   e4 = 2 pi i c dv'/dm0          (weight y_j, for m0)
#include "psf_device.hpp"
#include "psf_kernels.hpp"

namespace psf {

namespace {
// The per-sample factors use the hardware sine and cosine (expi_turns_hw):
// D_k stays within FP32 rounding of the FP64 mean, and D_k = 1 remains exact
// where every phase difference is 0.  The 16-pixel step factors of the
// records, raised to powers by the contraction's recurrence, keep the
// polynomial form.

// Channels per register chunk of bin_sums.  Four rather than eight: 70
// instead of 80 registers, seven waves per SIMD instead of six, which the
// loads of the sample loop need (factors of one source, D only: 0.156
// against 0.168 ms on the uniform-bin workload, 3.52 against 3.91 ms on the
// baseline-dependent bins of 1-8 channels); two channels re-read each
// time row too often (0.196 ms).
constexpr int kChanChunk = 4;

// Sums over one bin's samples: S = sum x e with e = exp(-2 pi i phi) and x
// the sample's window weight (1 without windows), the window sums of the bin
// along time (st) and channel (sc), and for the adjoint G_l = sum x g_l e and
// G_m = sum x g_m e with g = d phi / d(l0, m0).  The bin's channels are taken
// in chunks whose frequencies and channel windows sit in registers, so the
// only memory reads per time row are its uvw (and time window), loaded one
// row ahead.  Samples are summed time-major within a chunk.
struct BinSums {
  float sre, sim, glr, gli, gmr, gmi, st, sc;
};

template <bool kWin, bool kGrad>
__device__ __forceinline__ BinSums bin_sums(const ObsView& o, const BinRef& r, double l0, double m0, double Lw,
                                            double A_knu, double nu_k, double uc, double vc, double wc,
                                            double l0_n0, double m0_n0) {
#pragma clang fp contract(off)
  BinSums s{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const double* row = o.uvw + 3 * (static_cast<int64_t>(r.b) * o.n_t);
  const float* win_tb = kWin && o.win_t != nullptr ? o.win_t + static_cast<int64_t>(r.b) * o.n_t : nullptr;
  const float* win_cb = kWin && o.win_c != nullptr ? o.win_c + static_cast<int64_t>(r.b) * o.n_ch : nullptr;
  for (int cb = r.c0; cb < r.c1; cb += kChanChunk) {
    const int nch = min(kChanChunk, r.c1 - cb);
    double nu[kChanChunk];
    float xc[kChanChunk];
#pragma unroll
    for (int j = 0; j < kChanChunk; ++j) {
      const int c = cb + min(j, nch - 1);  // clamped: always a channel of the bin
      nu[j] = o.freq[c];
      xc[j] = kWin && win_cb != nullptr ? win_cb[c] : 1.f;
    }
    if constexpr (kWin) {
      // the window sums in channel and time order, from the loaded weights
#pragma unroll
      for (int j = 0; j < kChanChunk; ++j)
        if (j < nch) s.sc += xc[j];
    }
    double u = row[3 * r.t0], v = row[3 * r.t0 + 1], w = row[3 * r.t0 + 2];
    float xt = kWin && win_tb != nullptr ? win_tb[r.t0] : 1.f;
    for (int t = r.t0; t < r.t1; ++t) {
      const int tn = min(t + 1, r.t1 - 1);
      const double un = row[3 * tn], vn = row[3 * tn + 1], wn = row[3 * tn + 2];
      const float xtn = kWin && win_tb != nullptr ? win_tb[tn] : 1.f;
      if (kWin && cb == r.c0) s.st += xt;
      const double A_t = u * l0 + v * m0 + w * Lw;
#pragma unroll
      for (int j = 0; j < kChanChunk; ++j) {
        if (j < nch) {
          const double nu_c = nu[j];
          const double phi = (A_t * nu_c - A_knu) * kInvCLight;
          const cf32 e = expi_turns_hw(-phi);
          const float x = kWin ? xt * xc[j] : 1.f;
          if constexpr (kWin) {
            s.sre += x * e.re;
            s.sim += x * e.im;
          } else {
            s.sre += e.re;
            s.sim += e.im;
          }
          if constexpr (kGrad) {
            const double du = (u * nu_c - uc * nu_k) * kInvCLight;
            const double dv = (v * nu_c - vc * nu_k) * kInvCLight;
            const double dw = (w * nu_c - wc * nu_k) * kInvCLight;
            float gl = static_cast<float>(du - dw * l0_n0);
            float gm = static_cast<float>(dv - dw * m0_n0);
            if constexpr (kWin) {
              gl = x * gl;
              gm = x * gm;
            }
            // -2 pi i g e  =  2 pi g (e.im, -e.re); the 2 pi is applied by the caller
            s.glr += gl * e.im;
            s.gli -= gl * e.re;
            s.gmr += gm * e.im;
            s.gmi -= gm * e.re;
          }
        }
      }
      u = un;
      v = vn;
      w = wn;
      xt = xtn;
    }
  }
  return s;
}
}  // namespace

// The per-bin outputs from the bin's D (and, for the adjoint, its
// derivatives): D, the record the contraction streams (u', v' and the
// 16-pixel steps of both axes), c = W D, and the five adjoint coefficient
// vectors (only where the samples were summed, has_grad).
template <bool kGrad>
__device__ __forceinline__ void finish_bin(const ObsView& o, int64_t k, double l0, double m0, double n0, double dl,
                                           double dm, double nu_k, double uc, double vc, double wc, float dre,
                                           float dim, float dDl_re, float dDl_im, float dDm_re, float dDm_im,
                                           bool has_grad, float2* __restrict__ D_out, BinRec* __restrict__ rec_out,
                                           float2* __restrict__ c_out, float2* __restrict__ coef_out) {
#pragma clang fp contract(off)
  if (D_out != nullptr) D_out[k] = make_float2(dre, dim);
  const double s = nu_k * kInvCLight;
  const double u = uc * s, v = vc * s, w = wc * s;
  const double up = u - w * l0 / n0, vp = v - w * m0 / n0;
  if (rec_out != nullptr) {
    BinRec r;
    r.up = up;
    r.vp = vp;
    const cf32 sa = expi_turns(up * (16.0 * dl)), sb = expi_turns(vp * (16.0 * dm));
    r.step_a = make_float2(sa.re, sa.im);
    r.step_b = make_float2(sb.re, sb.im);
    // records and W D are streamed out (non-temporal stores: they exceed
    // every cache at the sizes that matter, 10.6 GB per source at K = 265M;
    // 5.35 against 5.58 ms per source there)
    static_assert(sizeof(BinRec) == 32 && offsetof(BinRec, vp) == 8 && offsetof(BinRec, step_a) == 16 &&
                      offsetof(BinRec, step_b) == 24,
                  "the record is stored as four 8-byte words");
    double* q = reinterpret_cast<double*>(rec_out + k);
    __builtin_nontemporal_store(r.up, q);
    __builtin_nontemporal_store(r.vp, q + 1);
    __builtin_nontemporal_store(__builtin_bit_cast(double, r.step_a), q + 2);
    __builtin_nontemporal_store(__builtin_bit_cast(double, r.step_b), q + 3);
  }
  const float W = o.W[k];
  const float cre = W * dre, cim = W * dim;
  if (c_out != nullptr)
    __builtin_nontemporal_store(__builtin_bit_cast(double, make_float2(cre, cim)), reinterpret_cast<double*>(c_out + k));
  if (kGrad && coef_out != nullptr && has_grad) {
    // 2 pi i c t = 2 pi t (-Im c, Re c) for real t.  All five vectors are
    // scaled by kAdjointScale (a power of two, exact) so that they stay in
    // the FP16 range of the split-FP16 contraction (|2 pi u' c| reaches a
    // few 1e5 on km baselines at GHz); the reduction undoes the scale.
    const double n03 = n0 * n0 * n0;
    const double two_pi = 6.283185307179586 * kAdjointScale;
    const float tu = static_cast<float>(two_pi * up), tv = static_cast<float>(two_pi * vp);
    const float t2 = static_cast<float>(-two_pi * w * (1.0 - m0 * m0) / n03);
    const float t3 = static_cast<float>(-two_pi * w * l0 * m0 / n03);
    const float t4 = static_cast<float>(-two_pi * w * (1.0 - l0 * l0) / n03);
    const int64_t K = o.K;
    const float Ws = W * static_cast<float>(kAdjointScale);
    coef_out[k] = make_float2(Ws * dDl_re - tu * -cim, Ws * dDl_im - tu * cre);
    coef_out[K + k] = make_float2(Ws * dDm_re - tv * -cim, Ws * dDm_im - tv * cre);
    coef_out[2 * K + k] = make_float2(t2 * -cim, t2 * cre);
    coef_out[3 * K + k] = make_float2(t3 * -cim, t3 * cre);
    coef_out[4 * K + k] = make_float2(t4 * -cim, t4 * cre);
  }
}

// One thread per bin.  Writes any subset of: D, record (u', v', c = W D),
// and the five adjoint coefficient vectors e0..e4 (coef_out, plane e at
// coef_out + e K).  When D_in is given the samples are not read: only the
// record is formed from the caller's D (no coefficients then).
//
// Several sources per launch: grid row y handles source y, whose direction
// is read from device memory at dirs + y * dir_stride (l0, m0 as the first
// two doubles) when dirs is given, and whose records start y * rec_stride
// elements into rec_out and c_out.
template <bool kGrad>
__global__ __launch_bounds__(256) void k_decorr(ObsView o, double l0, double m0, double dl, double dm,
                                                const double* __restrict__ dirs, int64_t dir_stride,
                                                int64_t rec_stride,
                                                const float2* __restrict__ D_in,
                                                float2* __restrict__ D_out,
                                                BinRec* __restrict__ rec_out,
                                                float2* __restrict__ c_out,
                                                float2* __restrict__ coef_out) {
  // No fused multiply-add in this kernel: the two products of the phase
  // difference must round alike so that identical rows cancel exactly.
#pragma clang fp contract(off)
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= o.K) return;
  if (dirs != nullptr) {
    l0 = dirs[blockIdx.y * dir_stride];
    m0 = dirs[blockIdx.y * dir_stride + 1];
    dl = dirs[blockIdx.y * dir_stride + 4];
    dm = dirs[blockIdx.y * dir_stride + 5];
  }
  if (rec_out != nullptr) rec_out += blockIdx.y * rec_stride;
  if (c_out != nullptr) c_out += blockIdx.y * rec_stride;
  const BinRef r = locate_bin(o.koff, o.tboff, o.bl_bin, o.n_bl, o.n_t, o.n_ch, k);
  const double n0 = sqrt(1.0 - l0 * l0 - m0 * m0);
  const double Lw = n0 - 1.0;
  const double nu_k = bin_freq(o.freq, r.c0, r.c1);
  const double uc = o.uvw_c[3 * r.tb + 0], vc = o.uvw_c[3 * r.tb + 1], wc = o.uvw_c[3 * r.tb + 2];

  float dre = 0.f, dim = 0.f;
  float dDl_re = 0.f, dDl_im = 0.f, dDm_re = 0.f, dDm_im = 0.f;
  if (D_in != nullptr) {
    const float2 d = D_in[k];
    dre = d.x;
    dim = d.y;
  } else {
    const double A_k = uc * l0 + vc * m0 + wc * Lw;
    const double A_knu = A_k * nu_k;
    const double l0_n0 = l0 / n0, m0_n0 = m0 / n0;
    float inv;
    BinSums bs;
    if (o.win_t != nullptr || o.win_c != nullptr) {
      // Windowed averaging: sample weight x = win_t[b][t] win_c[b][c], the
      // mean normalised by the window's sum over the bin (D = 0 for a
      // window that sums to 0).  Separable, so the normaliser is the
      // product of the two axis sums.
      bs = bin_sums<true, kGrad>(o, r, l0, m0, Lw, A_knu, nu_k, uc, vc, wc, l0_n0, m0_n0);
      const float norm = bs.st * bs.sc;
      inv = norm != 0.f ? 1.0f / norm : 0.f;
    } else {
      bs = bin_sums<false, kGrad>(o, r, l0, m0, Lw, A_knu, nu_k, uc, vc, wc, l0_n0, m0_n0);
      inv = 1.0f / static_cast<float>((r.t1 - r.t0) * (r.c1 - r.c0));
    }
    dre = bs.sre * inv;
    dim = bs.sim * inv;
    if constexpr (kGrad) {
      const float sc = 6.283185307179586f * inv;
      dDl_re = bs.glr * sc;
      dDl_im = bs.gli * sc;
      dDm_re = bs.gmr * sc;
      dDm_im = bs.gmi * sc;
    }
  }
  finish_bin<kGrad>(o, k, l0, m0, n0, dl, dm, nu_k, uc, vc, wc, dre, dim, dDl_re, dDl_im, dDm_re, dDm_im,
                    D_in == nullptr, D_out, rec_out, c_out, coef_out);
}

// Few long bins: one wave per bin.  When an observation has too few bins
// to fill the GPU with one lane each but many samples per bin (the host's
// choice, use_wave_bins), every wave takes one bin: lane l sums the bin's
// samples l, l + 64, ... in (time, channel) order, then the wave's partial
// sums are combined by a fixed butterfly of lane exchanges (deterministic,
// rounded in another order than the one-lane loop).  The per-sample phase
// is formed exactly as there (no fused multiply-add, so that identical rows
// still cancel exactly).  Four waves per block; source y of the launch in
// grid row y, as for k_decorr.
template <bool kGrad>
__global__ __launch_bounds__(256) void k_decorr_wave(ObsView o, double l0, double m0, double dl, double dm,
                                                     const double* __restrict__ dirs, int64_t dir_stride,
                                                     int64_t rec_stride, float2* __restrict__ D_out,
                                                     BinRec* __restrict__ rec_out, float2* __restrict__ c_out,
                                                     float2* __restrict__ coef_out) {
#pragma clang fp contract(off)
  const int64_t k = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (k >= o.K) return;  // the whole wave
  const int lane = threadIdx.x & 63;
  if (dirs != nullptr) {
    l0 = dirs[blockIdx.y * dir_stride];
    m0 = dirs[blockIdx.y * dir_stride + 1];
    dl = dirs[blockIdx.y * dir_stride + 4];
    dm = dirs[blockIdx.y * dir_stride + 5];
  }
  if (rec_out != nullptr) rec_out += blockIdx.y * rec_stride;
  if (c_out != nullptr) c_out += blockIdx.y * rec_stride;
  const BinRef r = locate_bin(o.koff, o.tboff, o.bl_bin, o.n_bl, o.n_t, o.n_ch, k);
  const double n0 = sqrt(1.0 - l0 * l0 - m0 * m0);
  const double Lw = n0 - 1.0;
  const double nu_k = bin_freq(o.freq, r.c0, r.c1);
  const double uc = o.uvw_c[3 * r.tb + 0], vc = o.uvw_c[3 * r.tb + 1], wc = o.uvw_c[3 * r.tb + 2];
  const double A_k = uc * l0 + vc * m0 + wc * Lw;
  const double A_knu = A_k * nu_k;
  const double l0_n0 = l0 / n0, m0_n0 = m0 / n0;
  const bool win = o.win_t != nullptr || o.win_c != nullptr;
  const int nc = r.c1 - r.c0, n = (r.t1 - r.t0) * nc;
  const double* rows = o.uvw + 3 * (static_cast<int64_t>(r.b) * o.n_t);
  float v[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // S re, im; G_l re, im; G_m re, im; window sum
  for (int idx = lane; idx < n; idx += 64) {
    const int t = r.t0 + idx / nc, c = r.c0 + idx % nc;
    const double u = rows[3 * t], vv = rows[3 * t + 1], w = rows[3 * t + 2];
    const double nu_c = o.freq[c];
    const double A_t = u * l0 + vv * m0 + w * Lw;
    const double phi = (A_t * nu_c - A_knu) * kInvCLight;
    const cf32 e = expi_turns_hw(-phi);
    float x = 1.f;
    if (win) {
      x = (o.win_t != nullptr ? o.win_t[static_cast<int64_t>(r.b) * o.n_t + t] : 1.f) *
          (o.win_c != nullptr ? o.win_c[static_cast<int64_t>(r.b) * o.n_ch + c] : 1.f);
      v[6] += x;
    }
    v[0] += x * e.re;
    v[1] += x * e.im;
    if constexpr (kGrad) {
      const double du = (u * nu_c - uc * nu_k) * kInvCLight;
      const double dv = (vv * nu_c - vc * nu_k) * kInvCLight;
      const double dw = (w * nu_c - wc * nu_k) * kInvCLight;
      const float gl = x * static_cast<float>(du - dw * l0_n0);
      const float gm = x * static_cast<float>(dv - dw * m0_n0);
      v[2] += gl * e.im;
      v[3] -= gl * e.re;
      v[4] += gm * e.im;
      v[5] -= gm * e.re;
    }
  }
#pragma unroll
  for (int q = 0; q < 7; ++q)
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off);
  if (lane != 0) return;
  const float inv = win ? (v[6] != 0.f ? 1.0f / v[6] : 0.f) : 1.0f / static_cast<float>(n);
  const float sc = 6.283185307179586f * inv;
  finish_bin<kGrad>(o, k, l0, m0, n0, dl, dm, nu_k, uc, vc, wc, v[0] * inv, v[1] * inv, v[2] * sc, v[3] * sc,
                    v[4] * sc, v[5] * sc, true, D_out, rec_out, c_out, coef_out);
}

// One wave per bin pays off when one lane per bin leaves the GPU mostly
// idle: fewer bins than 512 waves' worth and at least 64 samples per bin
// on average.
bool use_wave_bins(const ObsView& o) {
  const double samples = static_cast<double>(o.n_bl) * o.n_t * o.n_ch;
  return o.K > 0 && o.K < 512 * 64 && samples >= 64.0 * static_cast<double>(o.K);
}

hipError_t launch_decorr(const ObsView& o, double l0, double m0, double dl, double dm, const float2* D_in,
                         float2* D_out, BinRec* rec_out, float2* c_out, float2* coef_out, hipStream_t stream,
                         const double* dir) {
  const int threads = 256;
  const int64_t blocks = (o.K + threads - 1) / threads;
  if (D_in == nullptr && use_wave_bins(o)) {
    const dim3 g(static_cast<unsigned>((o.K + 3) / 4));
    if (coef_out != nullptr)
      hipLaunchKernelGGL(k_decorr_wave<true>, g, dim3(256), 0, stream, o, l0, m0, dl, dm, dir, int64_t(0),
                         int64_t(0), D_out, rec_out, c_out, coef_out);
    else
      hipLaunchKernelGGL(k_decorr_wave<false>, g, dim3(256), 0, stream, o, l0, m0, dl, dm, dir, int64_t(0),
                         int64_t(0), D_out, rec_out, c_out, nullptr);
    return hipGetLastError();
  }
  if (coef_out != nullptr && D_in == nullptr)
    hipLaunchKernelGGL(k_decorr<true>, dim3(static_cast<unsigned>(blocks)), dim3(threads), 0, stream, o, l0, m0,
                       dl, dm, dir, int64_t(0), int64_t(0), D_in, D_out, rec_out, c_out, coef_out);
  else
    hipLaunchKernelGGL(k_decorr<false>, dim3(static_cast<unsigned>(blocks)), dim3(threads), 0, stream, o, l0, m0,
                       dl, dm, dir, int64_t(0), int64_t(0), D_in, D_out, rec_out, c_out, nullptr);
  return hipGetLastError();
}

hipError_t launch_decorr_sources(const ObsView& o, const double* dirs, int64_t dir_stride, int n_src,
                                 BinRec* rec_out, float2* c_out, int64_t rec_stride, hipStream_t stream) {
  const int threads = 256;
  const int64_t blocks = (o.K + threads - 1) / threads;
  if (use_wave_bins(o)) {
    hipLaunchKernelGGL(k_decorr_wave<false>, dim3(static_cast<unsigned>((o.K + 3) / 4), static_cast<unsigned>(n_src)),
                       dim3(256), 0, stream, o, 0.0, 0.0, 0.0, 0.0, dirs, dir_stride, rec_stride, nullptr, rec_out,
                       c_out, nullptr);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_decorr<false>, dim3(static_cast<unsigned>(blocks), static_cast<unsigned>(n_src)), dim3(threads), 0,
                     stream, o, 0.0, 0.0, 0.0, 0.0, dirs, dir_stride, rec_stride, nullptr, nullptr, rec_out, c_out,
                     nullptr);
  return hipGetLastError();
}

}  // namespace psf

namespace psf {

// Method 1, the uv-plane approximation [section 3.1]: D_k replaced by
// sinc(dPsi/2) sinc(dPhi/2), dPsi = 2 pi du.(l0, m0) across the bin's time
// interval at its centre frequency, dPhi the same across its frequency
// interval at its centre time (2-D: w is dropped), sinc(x) = sin(x)/x.  A
// bin of n samples spaced by s covers n s: the change across it is n times
// the per-sample step, taken from the bin's first and last samples (from a
// neighbour for a one-sample bin; zero if the axis has one sample).  Only
// the bin's end rows are read, not its samples.  FP64; written as (D, 0).
__device__ __forceinline__ double sinc_of(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

__global__ __launch_bounds__(256) void k_decorr_sinc(ObsView o, double l0, double m0, float2* __restrict__ D_out) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= o.K) return;
  const BinRef r = locate_bin(o.koff, o.tboff, o.bl_bin, o.n_bl, o.n_t, o.n_ch, k);
  const double nu_k = bin_freq(o.freq, r.c0, r.c1);
  const double* row = o.uvw + 3 * (static_cast<int64_t>(r.b) * o.n_t);
  // per-sample step in time (metres)
  const int nt = r.t1 - r.t0;
  int ta, tb2;
  double div;
  if (nt > 1) {
    ta = r.t0;
    tb2 = r.t1 - 1;
    div = nt - 1;
  } else if (o.n_t > 1) {
    ta = r.t0 + 1 < o.n_t ? r.t0 : r.t0 - 1;
    tb2 = ta + 1;
    div = 1.0;
  } else {
    ta = tb2 = r.t0;
    div = 1.0;
  }
  const double su = (row[3 * tb2] - row[3 * ta]) / div, sv = (row[3 * tb2 + 1] - row[3 * ta + 1]) / div;
  // per-channel frequency step (Hz)
  const int nc = r.c1 - r.c0;
  double sf;
  if (nc > 1)
    sf = (o.freq[r.c1 - 1] - o.freq[r.c0]) / (nc - 1);
  else if (o.n_ch > 1)
    sf = r.c0 + 1 < o.n_ch ? o.freq[r.c0 + 1] - o.freq[r.c0] : o.freq[r.c0] - o.freq[r.c0 - 1];
  else
    sf = 0.0;
  const double pi = 3.141592653589793;
  const double x_t = pi * (nt * (su * l0 + sv * m0) * (nu_k * kInvCLight));
  const double uc = o.uvw_c[3 * r.tb], vc = o.uvw_c[3 * r.tb + 1];
  const double x_f = pi * ((uc * l0 + vc * m0) * (nc * sf * kInvCLight));
  D_out[k] = make_float2(static_cast<float>(sinc_of(x_t) * sinc_of(x_f)), 0.0f);
}

hipError_t launch_decorr_sinc(const ObsView& o, double l0, double m0, float2* D_out, hipStream_t stream) {
  const int threads = 256;
  const int64_t blocks = (o.K + threads - 1) / threads;
  hipLaunchKernelGGL(k_decorr_sinc, dim3(static_cast<unsigned>(blocks)), dim3(threads), 0, stream, o, l0, m0, D_out);
  return hipGetLastError();
}

}  // namespace psf
