// Adjoint of the patch with respect to the source direction (grid fixed).
//
// With G = dLoss/dP and the five coefficient vectors e0..e4 that k_decorr
// forms per bin (derivation in k_decorr.hip), write Q[e] for the patch of
// the same form as P with c_k replaced by e_k.  Then
//   dLoss/dl0 = sum_ij G_ij (Q0 + x_i Q2 + y_j Q3)_ij
//   dLoss/dm0 = sum_ij G_ij (Q1 + x_i Q3 + y_j Q4)_ij
// Each Q[e] runs through the same phase-factor generation and matrix-core
// contraction as the forward patch; k_grad_reduce forms the two sums in
// FP64 with a fixed reduction order.  The e vectors arrive scaled by
// kAdjointScale, which the reduction divides out.  Patches of up to
// 144 x 256 pixels in the split forms take the reverse-mode kernel of
// k_adjoint.hip instead (the same sums regrouped per visibility: two
// products of the patch's size per visibility rather than five patches).
#include <algorithm>

#include "psf_host.hpp"

namespace psf {

constexpr int kReduceThreads = 1024;

__global__ __launch_bounds__(kReduceThreads) void k_grad_reduce(const float* __restrict__ G,
                                                                const float* __restrict__ Pe, int nl, int nm,
                                                                double l_first, double dl, double l0,
                                                                double m_first, double dm, double m0,
                                                                const double* __restrict__ dir,
                                                                double* __restrict__ grad) {
  if (dir != nullptr) {  // direction and grid from device memory (psf_src layout)
    l0 = dir[0];
    m0 = dir[1];
    l_first = dir[2];
    m_first = dir[3];
    dl = dir[4];
    dm = dir[5];
  }
  const int64_t n = static_cast<int64_t>(nl) * nm;
  double gl = 0.0, gm = 0.0;
  for (int64_t p = threadIdx.x; p < n; p += kReduceThreads) {
    const int i = static_cast<int>(p / nm), j = static_cast<int>(p - static_cast<int64_t>(i) * nm);
    const double x = (l_first + i * dl) - l0, y = (m_first + j * dm) - m0;
    const double g = G[p];
    const double q0 = Pe[p], q1 = Pe[n + p], q2 = Pe[2 * n + p], q3 = Pe[3 * n + p], q4 = Pe[4 * n + p];
    gl += g * (q0 + x * q2 + y * q3);
    gm += g * (q1 + x * q3 + y * q4);
  }
  // fixed-order tree: butterfly within each wave, then across waves in LDS
  for (int o = 32; o > 0; o >>= 1) {
    gl += __shfl_xor(gl, o);
    gm += __shfl_xor(gm, o);
  }
  __shared__ double part[2][kReduceThreads / 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    part[0][wave] = gl;
    part[1][wave] = gm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sl = 0.0, sm = 0.0;
    for (int w = 0; w < kReduceThreads / 64; ++w) {
      sl += part[0][w];
      sm += part[1][w];
    }
    grad[0] = sl / kAdjointScale;
    grad[1] = sm / kAdjointScale;
  }
}

hipError_t launch_grad_reduce(const float* G, const float* Pe, int nl, int nm, double l_first, double dl,
                              double l0, double m_first, double dm, double m0, double* grad, hipStream_t stream,
                              const double* dir) {
  hipLaunchKernelGGL(k_grad_reduce, dim3(1), dim3(kReduceThreads), 0, stream, G, Pe, nl, nm, l_first, dl, l0,
                     m_first, dm, m0, dir, grad);
  return hipGetLastError();
}

namespace {
struct BackwardLayout {
  size_t rec, coef, partial, pe, adj, total;
};

// Gradients take split-FP16 products where the forward runs the mixed or
// stochastic form (whose statistical rounding bound is stated for patches
// only).
int backward_prec(int prec) { return prec == PSF_MIXED_FP16 || prec == PSF_SR_FP16 ? PSF_SPLIT_FP16 : prec; }

BackwardLayout backward_layout(const psf_obs* o, int n_src, const psf_src* h_srcs, int prec) {
  prec = backward_prec(prec);
  size_t partial = 0, pix = 0;
  for (int s = 0; s < n_src; ++s) {
    partial = std::max(partial, plan_patch(o, &h_srcs[s], prec, kTargetWorkgroups).partial_elems);
    pix = std::max(pix, static_cast<size_t>(h_srcs[s].nl) * h_srcs[s].nm);
  }
  BackwardLayout L;
  const size_t K = static_cast<size_t>(o->K);
  L.rec = 0;
  L.coef = L.rec + align_up(K * sizeof(BinRec), 256);
  L.partial = L.coef + align_up(5 * K * sizeof(float2), 256);
  L.pe = L.partial + align_up(partial * sizeof(float), 256);
  L.adj = L.pe + align_up(5 * pix * sizeof(float), 256);
  L.total = L.adj + align_up(adjoint_reverse_partial_bytes(), 256);
  return L;
}
}  // namespace

size_t backward_workspace(const psf_obs* o, int n_src, const psf_src* h_srcs, int prec) {
  return backward_layout(o, n_src, h_srcs, prec).total;
}

}  // namespace psf

namespace psf {
namespace {

// out[s][p] = flux[s] P[s][p]
__global__ __launch_bounds__(256) void k_flux_scale(const float* __restrict__ flux, const float* __restrict__ P,
                                                    int64_t npix, float* __restrict__ out) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (p >= npix) return;
  const int64_t e = static_cast<int64_t>(blockIdx.y) * npix + p;
  out[e] = flux[blockIdx.y] * P[e];
}

// One block per source: G = flux dL/dout (rounded from FP64) and
// dL/dflux = sum_p dL/dout P in FP64, reduced in a fixed order.
__global__ __launch_bounds__(256) void k_flux_backward(const float* __restrict__ flux, const float* __restrict__ P,
                                                       const float* __restrict__ gout, int64_t npix,
                                                       float* __restrict__ G, double* __restrict__ grad_flux) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * npix;
  const double f = flux[blockIdx.x];
  double acc = 0.0;
  for (int64_t p = threadIdx.x; p < npix; p += 256) {
    const double g = gout[base + p];
    G[base + p] = static_cast<float>(g * f);
    acc += g * static_cast<double>(P[base + p]);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) grad_flux[blockIdx.x] = ((part[0] + part[1]) + part[2]) + part[3];
}

int validate_flux(int32_t n_src, int64_t npix) {
  if (n_src < 1 || n_src > 65535) return fail(PSF_EINVAL, "n_src=%d outside 1..65535", n_src);
  if (npix < 1 || npix > (int64_t(1) << 31)) return fail(PSF_EINVAL, "npix=%lld outside 1..2^31", (long long)npix);
  return PSF_OK;
}

}  // namespace
}  // namespace psf

using namespace psf;

extern "C" int psf_flux_scale(int32_t n_src, int64_t npix, const float* flux, const float* P, float* out,
                              void* stream) {
  clear_error();
  int st;
  if ((st = validate_flux(n_src, npix)) != PSF_OK) return st;
  if (flux == nullptr || P == nullptr || out == nullptr) return fail(PSF_EINVAL, "flux, P or out is NULL");
  if ((st = check_device()) != PSF_OK) return st;
  hipLaunchKernelGGL(k_flux_scale, dim3(static_cast<unsigned>((npix + 255) / 256), n_src), dim3(256), 0,
                     static_cast<hipStream_t>(stream), flux, P, npix, out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PSF_OK : hip_fail(e, "k_flux_scale launch");
}

extern "C" int psf_flux_backward(int32_t n_src, int64_t npix, const float* flux, const float* P, const float* grad_out,
                                 float* G, double* grad_flux, void* stream) {
  clear_error();
  int st;
  if ((st = validate_flux(n_src, npix)) != PSF_OK) return st;
  if (flux == nullptr || P == nullptr || grad_out == nullptr || G == nullptr || grad_flux == nullptr)
    return fail(PSF_EINVAL, "a pointer argument is NULL");
  if ((st = check_device()) != PSF_OK) return st;
  hipLaunchKernelGGL(k_flux_backward, dim3(n_src), dim3(256), 0, static_cast<hipStream_t>(stream), flux, P, grad_out,
                     npix, G, grad_flux);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PSF_OK : hip_fail(e, "k_flux_backward launch");
}

extern "C" int psf_patch_backward(const psf_obs* obs, int32_t n_src, const psf_src* h_srcs, const psf_src* d_srcs,
                                  const float* G_all, int prec, double* grad_lm, void* ws, size_t ws_bytes,
                                  void* stream) {
  clear_error();
  int st;
  if ((st = validate_obs(obs)) != PSF_OK) return st;
  if ((st = validate_prec(prec)) != PSF_OK) return st;
  if ((st = reject_normalise(prec, "psf_patch_backward")) != PSF_OK) return st;
  prec = backward_prec(prec);
  if (n_src < 1 || h_srcs == nullptr) return fail(PSF_EINVAL, "need n_src >= 1 sources");
  for (int s = 0; s < n_src; ++s)
    if ((st = validate_src(&h_srcs[s], s)) != PSF_OK) return st;
  if (G_all == nullptr || grad_lm == nullptr) return fail(PSF_EINVAL, "G_all or grad_lm is NULL");
  const BackwardLayout L = backward_layout(obs, n_src, h_srcs, prec);
  if (ws == nullptr || ws_bytes < L.total)
    return fail(PSF_EWORKSPACE, "psf_patch_backward needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  if ((st = check_device()) != PSF_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* w = static_cast<uint8_t*>(ws);
  BinRec* rec = reinterpret_cast<BinRec*>(w + L.rec);
  float2* coef = reinterpret_cast<float2*>(w + L.coef);
  float* partial = reinterpret_cast<float*>(w + L.partial);
  float* pe = reinterpret_cast<float*>(w + L.pe);
  double* adj = reinterpret_cast<double*>(w + L.adj);
  const int64_t K = obs->K;
  for (int n = 0; n < n_src; ++n) {
    const psf_src& src = h_srcs[n];
    // directions and grids from the device array when given (read at run
    // time, so a captured call replays for new directions)
    const double* dir = d_srcs != nullptr ? reinterpret_cast<const double*>(d_srcs + n) : nullptr;
    const int64_t pix = static_cast<int64_t>(src.nl) * src.nm;
    hipError_t e;
    if (K > 0) {
      e = launch_decorr(view(obs), src.l0, src.m0, src.dl, src.dm, nullptr, nullptr, rec, nullptr, coef, s, dir);
      if (e != hipSuccess) return hip_fail(e, "k_decorr launch");
    }
    if (adjoint_reverse_ok(prec, obs, src)) {
      e = launch_adjoint_reverse(obs, src, prec, rec, coef, G_all + src.out_off, adj, grad_lm + 2 * n, s, dir);
      if (e != hipSuccess) return hip_fail(e, "k_adjoint launch");
      continue;
    }
    const PatchPlan plan = plan_patch(obs, &src, prec, kTargetWorkgroups);
    for (int q = 0; q < 5; ++q)
      if ((st = contract(obs, &src, plan, prec, rec, coef + q * K, partial, pe + q * pix, s, dir)) != PSF_OK)
        return st;
    e = launch_grad_reduce(G_all + src.out_off, pe, src.nl, src.nm, src.l_first, src.dl, src.l0, src.m_first,
                           src.dm, src.m0, grad_lm + 2 * n, s, dir);
    if (e != hipSuccess) return hip_fail(e, "k_grad_reduce launch");
  }
  return PSF_OK;
}
