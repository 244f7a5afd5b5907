// The patch with the exact w phase [section 2.1: the visibility relation
// keeps the w (n - 1) term]: relative to the source the imaging phase of bin
// k at pixel (i, j) is u x_i + v y_j + w (n_ij - n0), which is the
// linearised phase u' x_i + v' y_j (u' = u - w l0/n0, v' = v - w m0/n0)
// plus w q_ij with
//   q_ij = n_ij - n0 + (l0 x_i + m0 y_j) / n0 .
// n is concave on the sky, so q <= 0 (0 at the source) and its minimum over
// the patch sits on a corner of the grid.
//
// The extra factor exp(2 pi i w_k q_ij) couples k and (i, j), so it is
// expanded into matrix-core contractions of the linearised form.  With
// s >= max |w_k|, z_k = w_k / s in [-1, 1], y_ij = 2 pi s q_ij in [y_lo, 0],
// centre ybar = y_lo / 2 and delta_ij = y_ij - ybar in [-Y, Y], Y = -y_lo/2:
//   exp(i z y) = exp(i z ybar) sum_r (i z)^r delta^r / r!
// so   P = sum_{r=0..R} (delta_ij / Y)^r P^(r),
// where P^(r) is the linearised patch with coefficients
//   c^(r)_k = W_k D_k exp(i z_k ybar) (i z_k)^r Y^r / r! .
// The pixel weights (delta / Y)^r lie in [-1, 1] and the coefficients
// shrink with r, so no term leaves the FP16 range of the split-FP16 form.
// R is the smallest order whose truncation bound Y^(R+1)/(R+1)! is at most
// kTruncation (1e-7 of the coefficient sum, below the contraction's own
// rounding); Y is limited to kMaxY so that the terms (together up to e^Y of
// the patch) do not amplify the contraction's rounding past 1e-5.
#include <cmath>

#include "psf_device.hpp"
#include "psf_host.hpp"

namespace psf {

namespace {

constexpr double kMaxY = 2.0;
constexpr double kTruncation = 1e-7;
constexpr int kMaxOrder = 40;

// s = max |w_c| over the time-bin centres times the largest channel
// frequency: an upper bound of |w_k| (wavelengths) for every bin.  Two
// stages: kWmaxBlocks partial maxima (grid-stride), then one block.
constexpr int kWmaxBlocks = 256;

__device__ __forceinline__ void block_max2(double& w, double& f) {
  __shared__ double sw[256], sf[256];
  sw[threadIdx.x] = w;
  sf[threadIdx.x] = f;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (static_cast<int>(threadIdx.x) < o) {
      sw[threadIdx.x] = fmax(sw[threadIdx.x], sw[threadIdx.x + o]);
      sf[threadIdx.x] = fmax(sf[threadIdx.x], sf[threadIdx.x + o]);
    }
    __syncthreads();
  }
  w = sw[0];
  f = sf[0];
}

__global__ __launch_bounds__(256) void k_wmax_partial(const double* __restrict__ uvw_c, int64_t n_tb,
                                                     const double* __restrict__ freq, int n_ch,
                                                     double* __restrict__ part) {
  double w = 0.0, f = 0.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; t < n_tb; t += stride)
    w = fmax(w, fabs(uvw_c[3 * t + 2]));
  for (int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; c < n_ch; c += stride)
    f = fmax(f, fabs(freq[c]));
  block_max2(w, f);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = w;
    part[2 * blockIdx.x + 1] = f;
  }
}

__global__ __launch_bounds__(256) void k_wmax_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  double w = 0.0, f = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    w = fmax(w, part[2 * b]);
    f = fmax(f, part[2 * b + 1]);
  }
  block_max2(w, f);
  if (threadIdx.x == 0) out[0] = w * f * kInvCLight;
}

// Per bin: z_k = w_k / s and c~_k = c_k exp(i z_k ybar) (FP64 phase).
__global__ __launch_bounds__(256) void k_fullw_prep(ObsView o, const float2* __restrict__ c, double inv_s,
                                                    double ybar, float2* __restrict__ ct, float* __restrict__ z) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= o.K) return;
  const BinRef r = locate_bin(o.koff, o.tboff, o.bl_bin, o.n_bl, o.n_t, o.n_ch, k);
  const double w = o.uvw_c[3 * r.tb + 2] * bin_freq(o.freq, r.c0, r.c1) * kInvCLight;
  const double zk = w * inv_s;
  double sn, cs;
  sincos(zk * ybar, &sn, &cs);
  const float2 ck = c[k];
  const float cr = static_cast<float>(cs), ci = static_cast<float>(sn);
  ct[k] = make_float2(ck.x * cr - ck.y * ci, ck.x * ci + ck.y * cr);
  z[k] = static_cast<float>(zk);
}

// c^(r)_k = c~_k (i z_k)^r scale, scale = Y^r / r!
__global__ __launch_bounds__(256) void k_fullw_coef(const float2* __restrict__ ct, const float* __restrict__ z,
                                                    int64_t K, int r, float scale, float2* __restrict__ out) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= K) return;
  float p = scale;
  const float zk = z[k];
  for (int q = 0; q < r; ++q) p *= zk;
  const float2 a = ct[k];
  float2 v;
  switch (r & 3) {
    case 0: v = make_float2(a.x, a.y); break;
    case 1: v = make_float2(-a.y, a.x); break;
    case 2: v = make_float2(-a.x, -a.y); break;
    default: v = make_float2(a.y, -a.x); break;
  }
  out[k] = make_float2(v.x * p, v.y * p);
}

struct GridArgs {
  double l_first, m_first, dl, dm, l0, m0, n0;
  double two_pi_s, ybar, inv_Y;
  int nl, nm;
};

// q = n - n0 + (l0 x + m0 y)/n0 with n - n0 = (n^2 - n0^2)/(n + n0) written
// without the cancellation of two square roots near 1.
__host__ __device__ inline double q_of(double l0, double m0, double n0, double x, double y) {
  const double l = l0 + x, m = m0 + y;
  const double n = sqrt(1.0 - l * l - m * m);
  const double dn = -(x * (2.0 * l0 + x) + y * (2.0 * m0 + y)) / (n + n0);
  return dn + (l0 * x + m0 * y) / n0;
}

// out (+)= (delta_ij / Y)^r P^(r)_ij
__global__ __launch_bounds__(256) void k_fullw_accum(GridArgs g, int r, const float* __restrict__ Pr,
                                                     float* __restrict__ out) {
  const int64_t n = static_cast<int64_t>(g.nl) * g.nm;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  if (r == 0) {
    out[p] = Pr[p];
    return;
  }
  const int i = static_cast<int>(p / g.nm), j = static_cast<int>(p - static_cast<int64_t>(i) * g.nm);
  const double x = (g.l_first + i * g.dl) - g.l0, y = (g.m_first + j * g.dm) - g.m0;
  const double d = (g.two_pi_s * q_of(g.l0, g.m0, g.n0, x, y) - g.ybar) * g.inv_Y;
  double dr = 1.0;
  for (int q = 0; q < r; ++q) dr *= d;
  out[p] += static_cast<float>(dr) * Pr[p];
}

struct FullwLayout {
  size_t ct, z, cr, Pr, s, total;
};

FullwLayout fullw_layout(const psf_obs* o, const psf_src* src, const PatchPlan& plan) {
  FullwLayout L;
  const size_t K = static_cast<size_t>(o->K);
  L.ct = align_up(patch_workspace(o, plan), 256);
  L.z = L.ct + align_up(K * sizeof(float2), 256);
  L.cr = L.z + align_up(K * sizeof(float), 256);
  L.Pr = L.cr + align_up(K * sizeof(float2), 256);
  L.s = L.Pr + align_up(static_cast<size_t>(src->nl) * src->nm * sizeof(float), 256);
  L.total = L.s + align_up((2 * kWmaxBlocks + 1) * sizeof(double), 256);
  return L;
}

// Grid corners inside the sky; q_lo = min of q over the corners (<= 0).
int fullw_grid(const psf_src* s, double* q_lo) {
  const double n0 = std::sqrt(1.0 - s->l0 * s->l0 - s->m0 * s->m0);
  const double ls[2] = {s->l_first, s->l_first + (s->nl - 1) * s->dl};
  const double ms[2] = {s->m_first, s->m_first + (s->nm - 1) * s->dm};
  double lo = 0.0;
  for (double l : ls)
    for (double m : ms) {
      if (!(l * l + m * m < 1.0)) return fail(PSF_EINVAL, "patch corner (%g, %g) outside the sky", l, m);
      lo = std::fmin(lo, q_of(s->l0, s->m0, n0, l - s->l0, m - s->m0));
    }
  *q_lo = lo;
  return PSF_OK;
}

}  // namespace

size_t fullw_workspace(const psf_obs* o, int n_src, const psf_src* h_srcs, int prec) {
  size_t need = 0;
  for (int s = 0; s < n_src; ++s) {
    const PatchPlan plan = plan_patch(o, &h_srcs[s], prec, kTargetWorkgroups);
    need = std::max(need, fullw_layout(o, &h_srcs[s], plan).total);
  }
  return need;
}

}  // namespace psf

using namespace psf;

extern "C" {

int psf_patch_fullw(const psf_obs* obs, const psf_src* h_src, int prec, float* P, int32_t* n_terms, void* ws,
                    size_t ws_bytes, void* stream) {
  clear_error();
  int st;
  if ((st = validate_obs(obs)) != PSF_OK) return st;
  if ((st = validate_src(h_src, 0)) != PSF_OK) return st;
  if ((st = validate_prec(prec)) != PSF_OK) return st;
  if ((st = reject_normalise(prec, "psf_patch_fullw")) != PSF_OK) return st;
  if (P == nullptr) return fail(PSF_EINVAL, "P is NULL");
  double q_lo = 0.0;
  if ((st = fullw_grid(h_src, &q_lo)) != PSF_OK) return st;
  const PatchPlan plan = plan_patch(obs, h_src, prec, kTargetWorkgroups);
  const FullwLayout L = fullw_layout(obs, h_src, plan);
  if (ws == nullptr || ws_bytes < L.total)
    return fail(PSF_EWORKSPACE, "psf_patch_fullw needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  if ((st = check_device()) != PSF_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* w = static_cast<uint8_t*>(ws);
  BinRec* rec = reinterpret_cast<BinRec*>(w);
  float2* c = reinterpret_cast<float2*>(w + align_up(static_cast<size_t>(obs->K) * sizeof(BinRec), 256));
  float* partial = reinterpret_cast<float*>(reinterpret_cast<uint8_t*>(c) +
                                            align_up(static_cast<size_t>(obs->K) * sizeof(float2), 256));
  float2* ct = reinterpret_cast<float2*>(w + L.ct);
  float* z = reinterpret_cast<float*>(w + L.z);
  float2* cr = reinterpret_cast<float2*>(w + L.cr);
  float* Pr = reinterpret_cast<float*>(w + L.Pr);
  double* d_s = reinterpret_cast<double*>(w + L.s);

  hipError_t e = hipSuccess;
  double smax = 0.0;
  if (obs->K > 0) {
    e = launch_decorr(view(obs), h_src->l0, h_src->m0, h_src->dl, h_src->dm, nullptr, nullptr, rec, c, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "k_decorr launch");
    double* part = d_s + 1;
    hipLaunchKernelGGL(k_wmax_partial, dim3(kWmaxBlocks), dim3(256), 0, s, obs->uvw_c_m, obs->n_tb, obs->freq_hz,
                       obs->n_ch, part);
    hipLaunchKernelGGL(k_wmax_final, dim3(1), dim3(256), 0, s, part, kWmaxBlocks, d_s);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_wmax launch");
    if ((e = hipMemcpyAsync(&smax, d_s, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return hip_fail(e, "w bound read-back");
  }
  // Expansion order from the range of y = 2 pi s q over the patch.
  const double y_lo = 2.0 * M_PI * smax * q_lo;
  const double ybar = 0.5 * y_lo, Y = -0.5 * y_lo;
  if (!(Y <= kMaxY))
    return fail(PSF_EINVAL, "non-linear w phase spans %.3g rad over the patch (limit %.3g): patch too wide", 2.0 * Y,
                2.0 * kMaxY);
  int R = 0;
  double bound = Y;  // Y^(R+1)/(R+1)!
  while (bound > kTruncation && R < kMaxOrder) {
    ++R;
    bound *= Y / (R + 1);
  }
  if (n_terms != nullptr) *n_terms = R + 1;
  if (obs->K == 0 || smax == 0.0 || R == 0) return contract(obs, h_src, plan, prec, rec, c, partial, P, s);

  const unsigned kb = static_cast<unsigned>((obs->K + 255) / 256);
  hipLaunchKernelGGL(k_fullw_prep, dim3(kb), dim3(256), 0, s, view(obs), c, 1.0 / smax, ybar, ct, z);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_fullw_prep launch");
  GridArgs g;
  g.l_first = h_src->l_first;
  g.m_first = h_src->m_first;
  g.dl = h_src->dl;
  g.dm = h_src->dm;
  g.l0 = h_src->l0;
  g.m0 = h_src->m0;
  g.n0 = std::sqrt(1.0 - h_src->l0 * h_src->l0 - h_src->m0 * h_src->m0);
  g.two_pi_s = 2.0 * M_PI * smax;
  g.ybar = ybar;
  g.inv_Y = 1.0 / Y;
  g.nl = h_src->nl;
  g.nm = h_src->nm;
  const int64_t npix = static_cast<int64_t>(h_src->nl) * h_src->nm;
  const unsigned pb = static_cast<unsigned>((npix + 255) / 256);
  double scale = 1.0;  // Y^r / r!
  for (int r = 0; r <= R; ++r) {
    if (r > 0) scale *= Y / r;
    hipLaunchKernelGGL(k_fullw_coef, dim3(kb), dim3(256), 0, s, ct, z, obs->K, r, static_cast<float>(scale), cr);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_fullw_coef launch");
    if ((st = contract(obs, h_src, plan, prec, rec, cr, partial, Pr, s)) != PSF_OK) return st;
    hipLaunchKernelGGL(k_fullw_accum, dim3(pb), dim3(256), 0, s, g, r, Pr, P);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_fullw_accum launch");
  }
  return PSF_OK;
}

}  // extern "C"
