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
#include "psf_device.hpp"
#include "psf_kernels.hpp"

namespace psf {

// One thread per bin.  Writes any subset of: D, record (u', v', c = W D),
// and the two derivatives.  When D_in is given the samples are not read:
// only the record is formed from the caller's D.
__global__ __launch_bounds__(256) void k_decorr(ObsView o, double l0, double m0,
                                                const float2* __restrict__ D_in,
                                                float2* __restrict__ D_out,
                                                double2* __restrict__ uvp_out,
                                                float2* __restrict__ c_out,
                                                float2* __restrict__ dDl_out,
                                                float2* __restrict__ dDm_out) {
  // No fused multiply-add in this kernel: the two products of the phase
  // difference must round alike so that identical rows cancel exactly.
#pragma clang fp contract(off)
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= o.K) return;
  const BinRef r = locate_bin(o.koff, o.tboff, o.bl_bin, o.n_bl, o.n_t, o.n_ch, k);
  const double n0 = sqrt(1.0 - l0 * l0 - m0 * m0);
  const double Lw = n0 - 1.0;
  const double nu_k = bin_freq(o.freq, r.c0, r.c1);
  const double uc = o.uvw_c[3 * r.tb + 0], vc = o.uvw_c[3 * r.tb + 1], wc = o.uvw_c[3 * r.tb + 2];

  float dre = 0.f, dim = 0.f;
  if (D_in != nullptr) {
    const float2 d = D_in[k];
    dre = d.x;
    dim = d.y;
  } else {
    const bool grad = dDl_out != nullptr;
    const double A_k = uc * l0 + vc * m0 + wc * Lw;
    const double A_knu = A_k * nu_k;
    float sre = 0.f, sim = 0.f;
    float glr = 0.f, gli = 0.f, gmr = 0.f, gmi = 0.f;
    const double* row = o.uvw + 3 * (static_cast<int64_t>(r.b) * o.n_t);
    for (int t = r.t0; t < r.t1; ++t) {
      const double u = row[3 * t + 0], v = row[3 * t + 1], w = row[3 * t + 2];
      const double A_t = u * l0 + v * m0 + w * Lw;
      for (int c = r.c0; c < r.c1; ++c) {
        const double nu = o.freq[c];
        const double phi = (A_t * nu - A_knu) * kInvCLight;
        const cf32 e = expi_turns(-phi);
        sre += e.re;
        sim += e.im;
        if (grad) {
          const double du = (u * nu - uc * nu_k) * kInvCLight;
          const double dv = (v * nu - vc * nu_k) * kInvCLight;
          const double dw = (w * nu - wc * nu_k) * kInvCLight;
          const float gl = static_cast<float>(du - dw * l0 / n0);
          const float gm = static_cast<float>(dv - dw * m0 / n0);
          // -2 pi i g e  =  2 pi g (e.im, -e.re)
          glr += gl * e.im; gli -= gl * e.re;
          gmr += gm * e.im; gmi -= gm * e.re;
        }
      }
    }
    const float inv_n = 1.0f / static_cast<float>((r.t1 - r.t0) * (r.c1 - r.c0));
    dre = sre * inv_n;
    dim = sim * inv_n;
    if (grad) {
      const float s = 6.283185307179586f * inv_n;
      dDl_out[k] = make_float2(glr * s, gli * s);
      dDm_out[k] = make_float2(gmr * s, gmi * s);
    }
  }
  if (D_out != nullptr) D_out[k] = make_float2(dre, dim);
  if (uvp_out != nullptr) {
    const double s = nu_k * kInvCLight;
    const double u = uc * s, v = vc * s, w = wc * s;
    uvp_out[k] = make_double2(u - w * l0 / n0, v - w * m0 / n0);
  }
  if (c_out != nullptr) {
    const float W = o.W[k];
    c_out[k] = make_float2(W * dre, W * dim);
  }
}

hipError_t launch_decorr(const ObsView& o, double l0, double m0, const float2* D_in, float2* D_out,
                         double2* uvp_out, float2* c_out, float2* dDl_out, float2* dDm_out,
                         hipStream_t stream) {
  const int threads = 256;
  const int64_t blocks = (o.K + threads - 1) / threads;
  hipLaunchKernelGGL(k_decorr, dim3(static_cast<unsigned>(blocks)), dim3(threads), 0, stream, o, l0,
                     m0, D_in, D_out, uvp_out, c_out, dDl_out, dDm_out);
  return hipGetLastError();
}

}  // namespace psf
