// Method 2, the image-plane approximation [section 3.2]: every baseline is
// given the same decorrelation, pixelised over the uv plane from a
// fringe-rate model [Algorithm 1], and applied to the effective PSF (the
// PSF at the phase centre, section 2.2) as a product in the Fourier domain:
//   P^_d(l0, .) = F^-1 { F{P_eff} D^(l0) } .
// The effective PSF is computed once (psf_method2_spectrum: the patch
// contraction at l0 = m0 = 0, where every D_k is exactly 1, then a 2-D FFT);
// each source then costs one pointwise product and one inverse 2-D FFT
// (psf_method2_patch, up to kChunk sources per launch).
//
// Grid: N x N (N a power of two), pixel i at offset (i - N/2) cell; uv cell
// a at frequency a' du, du = 1/(N cell), with a' = a for a < N/2 and a - N
// otherwise (the DFT's own order, in which the spectrum is kept).
// Fringe-rate model: a circular track of radius |u0| turning at omega_E, so
//   dPsi = 2 pi omega_E (-v0 l0 + u0 m0) dt,  dPhi = 2 pi (dnu/nu) |l0| |u0|,
//   D^ = sinc(dPsi/2) sinc(dPhi/2).
//
// FFTs: radix-2 Stockham (self-sorting) on one line per workgroup, held in
// LDS (two buffers of N complex floats), FP32 with twiddles exp(+-2 pi i
// p/n) from sincospi of an exactly representable argument.
#include <algorithm>
#include <cmath>

#include "psf_host.hpp"

namespace psf {

namespace {

constexpr double kOmegaEarth = 7.2921150e-5;  // rad / s, sidereal
constexpr int kChunk = 16;                    // sources per launch
constexpr int kFftThreads = 256;

__global__ __launch_bounds__(kFftThreads) void k_fft_lines(float2* __restrict__ data, int N, int logN,
                                                           int64_t elem_stride, int64_t line_stride,
                                                           int64_t batch_stride, float sign) {
  extern __shared__ float2 lds[];
  float2* base = data + blockIdx.y * batch_stride + blockIdx.x * line_stride;
  for (int n = threadIdx.x; n < N; n += kFftThreads) lds[n] = base[n * elem_stride];
  __syncthreads();
  int cur = 0;
  for (int pass = 0; pass < logN; ++pass) {
    const int n_sz = N >> pass, m = n_sz >> 1, ls = pass;  // stride s = 2^pass
    const float2* in = lds + cur * N;
    float2* out = lds + (cur ^ 1) * N;
    for (int t = threadIdx.x; t < (N >> 1); t += kFftThreads) {
      const int p = t >> ls, q = t - (p << ls);
      float sn, cs;
      sincospif(sign * 2.0f * static_cast<float>(p) / static_cast<float>(n_sz), &sn, &cs);
      const float2 a = in[q + (p << ls)];
      const float2 b = in[q + ((p + m) << ls)];
      out[q + ((2 * p) << ls)] = make_float2(a.x + b.x, a.y + b.y);
      const float dx = a.x - b.x, dy = a.y - b.y;
      out[q + ((2 * p + 1) << ls)] = make_float2(dx * cs - dy * sn, dx * sn + dy * cs);
    }
    __syncthreads();
    cur ^= 1;
  }
  for (int n = threadIdx.x; n < N; n += kFftThreads) base[n * elem_stride] = lds[cur * N + n];
}

// Centred real image (row pitch `pitch` >= N) -> DFT order complex:
// buf[(i + N/2) % N][(j + N/2) % N] = P[i][j].
__global__ __launch_bounds__(256) void k_m2_load(const float* __restrict__ P, int pitch, float2* __restrict__ buf,
                                                 int N) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= static_cast<int64_t>(N) * N) return;
  const int i = static_cast<int>(e / N), j = static_cast<int>(e - static_cast<int64_t>(i) * N);
  const int h = N >> 1, msk = N - 1;
  buf[static_cast<int64_t>((i + h) & msk) * N + ((j + h) & msk)] =
      make_float2(P[static_cast<int64_t>(i) * pitch + j], 0.0f);
}

struct Dirs {
  double l0[kChunk], m0[kChunk];
};

// work[s][a][b] = S[a][b] D^(a' du, b' du; l0_s, m0_s); the direction of
// a one-source launch read from device memory (l0, m0 at ddir) when ddir
// is not null.
__global__ __launch_bounds__(256) void k_m2_dhat(const float2* __restrict__ S, float2* __restrict__ work, int N,
                                                 double du, double dt, double frac_bw, Dirs d,
                                                 const double* __restrict__ ddir) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t NN = static_cast<int64_t>(N) * N;
  if (e >= NN) return;
  const int s = blockIdx.y;
  const int a = static_cast<int>(e / N), b = static_cast<int>(e - static_cast<int64_t>(a) * N);
  const double u0 = (a < N / 2 ? a : a - N) * du, v0 = (b < N / 2 ? b : b - N) * du;
  const double l0 = ddir != nullptr ? ddir[0] : d.l0[s], m0 = ddir != nullptr ? ddir[1] : d.m0[s];
  const double hpsi = M_PI * kOmegaEarth * (-v0 * l0 + u0 * m0) * dt;  // dPsi / 2
  const double hphi = M_PI * frac_bw * sqrt(l0 * l0 + m0 * m0) * sqrt(u0 * u0 + v0 * v0);
  const double sp = hpsi == 0.0 ? 1.0 : sin(hpsi) / hpsi;
  const double sf = hphi == 0.0 ? 1.0 : sin(hphi) / hphi;
  const float dh = static_cast<float>(sp * sf);
  const float2 v = S[e];
  work[s * NN + e] = make_float2(v.x * dh, v.y * dh);
}

// P[s][i][j] = Re work[s][(i + N/2) % N][(j + N/2) % N] / N^2
__global__ __launch_bounds__(256) void k_m2_store(const float2* __restrict__ work, float* __restrict__ P, int N,
                                                  float scale) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t NN = static_cast<int64_t>(N) * N;
  if (e >= NN) return;
  const int s = blockIdx.y;
  const int i = static_cast<int>(e / N), j = static_cast<int>(e - static_cast<int64_t>(i) * N);
  const int h = N >> 1, msk = N - 1;
  P[s * NN + e] = work[s * NN + static_cast<int64_t>((i + h) & msk) * N + ((j + h) & msk)].x * scale;
}

int log2_exact(int N) {
  int l = 0;
  while ((1 << l) < N) ++l;
  return (1 << l) == N ? l : -1;
}

int validate_grid(int32_t N, double cell) {
  if (N < 16 || N > 4096 || log2_exact(N) < 0) return fail(PSF_EINVAL, "N=%d must be a power of two in 16..4096", N);
  if (!(cell > 0.0) || !std::isfinite(cell) || cell * N / 2 >= 1.0)
    return fail(PSF_EINVAL, "cell %g must be positive and the grid inside the sky", cell);
  return PSF_OK;
}

// 2-D FFT of n_batch N x N complex arrays in place: rows, then columns.
int fft2(float2* data, int N, int n_batch, float sign, hipStream_t s) {
  const int logN = log2_exact(N);
  const size_t lds = 2 * static_cast<size_t>(N) * sizeof(float2);
  const int64_t NN = static_cast<int64_t>(N) * N;
  hipLaunchKernelGGL(k_fft_lines, dim3(N, n_batch), dim3(kFftThreads), lds, s, data, N, logN, int64_t(1),
                     int64_t(N), NN, sign);
  hipLaunchKernelGGL(k_fft_lines, dim3(N, n_batch), dim3(kFftThreads), lds, s, data, N, logN, int64_t(N),
                     int64_t(1), NN, sign);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? PSF_OK : hip_fail(e, "k_fft_lines launch");
}

// The grid the effective PSF is contracted on: offsets -N/2 .. N/2 - 1, or
// -N/2 .. N/2 (one more row and column, dropped when loaded) where N + 1 is
// one of the patch sizes with a tuned tile family (65, 129, 257).
psf_src effective_grid(int32_t N, double cell) {
  psf_src g{};
  g.l0 = g.m0 = 0.0;
  g.l_first = g.m_first = -(N / 2) * cell;
  g.dl = g.dm = cell;
  g.nl = g.nm = (N == 64 || N == 128 || N == 256) ? N + 1 : N;
  g.out_off = 0;
  return g;
}

struct SpectrumLayout {
  size_t Peff, total;
};

SpectrumLayout spectrum_layout(const psf_obs* o, const PatchPlan& plan, int32_t N) {
  SpectrumLayout L;
  L.Peff = align_up(patch_workspace(o, plan), 256);
  L.total = L.Peff + align_up(static_cast<size_t>(N + 1) * (N + 1) * sizeof(float), 256);
  return L;
}

size_t patch_m2_workspace(int32_t N, int32_t n_src) {
  return static_cast<size_t>(std::min(n_src, kChunk)) * N * N * sizeof(float2);
}

}  // namespace

// One Method-2 patch whose direction (l0, m0) is read from device memory
// when the kernels run (the arguments validated by the caller; work holds
// N^2 complex values).
int method2_patch_device_dir(int32_t N, double cell, const float* S, const double* d_dir, double dt_bin,
                             double dnu_bin, double nu, float* P, float2* work, hipStream_t s) {
  const int64_t NN = static_cast<int64_t>(N) * N;
  const unsigned nb = static_cast<unsigned>((NN + 255) / 256);
  const double du = 1.0 / (N * cell);
  hipLaunchKernelGGL(k_m2_dhat, dim3(nb, 1), dim3(256), 0, s, reinterpret_cast<const float2*>(S), work, N, du,
                     dt_bin, dnu_bin / nu, Dirs{}, d_dir);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_m2_dhat launch");
  int st;
  if ((st = fft2(work, N, 1, 1.0f, s)) != PSF_OK) return st;
  hipLaunchKernelGGL(k_m2_store, dim3(nb, 1), dim3(256), 0, s, work, P, N,
                     static_cast<float>(1.0 / static_cast<double>(NN)));
  e = hipGetLastError();
  return e == hipSuccess ? PSF_OK : hip_fail(e, "k_m2_store launch");
}

}  // namespace psf

using namespace psf;

extern "C" {

int psf_method2_workspace_bytes(const psf_obs* obs, int32_t N, int prec, int32_t n_src, size_t* out) {
  clear_error();
  int st;
  if ((st = validate_obs(obs)) != PSF_OK) return st;
  if ((st = validate_prec(prec)) != PSF_OK) return st;
  if ((st = reject_normalise(prec, "psf_method2")) != PSF_OK) return st;
  if ((st = validate_grid(N, 1e-6)) != PSF_OK) return st;
  if (n_src < 0) return fail(PSF_EINVAL, "n_src < 0");
  if (out == nullptr) return fail(PSF_EINVAL, "out is NULL");
  const psf_src g = effective_grid(N, 1e-6);
  const PatchPlan plan = plan_patch(obs, &g, prec, kTargetWorkgroups);
  *out = std::max(spectrum_layout(obs, plan, N).total, patch_m2_workspace(N, std::max(n_src, 1)));
  return PSF_OK;
}

int psf_method2_spectrum(const psf_obs* obs, int32_t N, double cell, int prec, float* S, void* ws, size_t ws_bytes,
                         void* stream) {
  clear_error();
  int st;
  if ((st = validate_obs(obs)) != PSF_OK) return st;
  if ((st = validate_prec(prec)) != PSF_OK) return st;
  if ((st = reject_normalise(prec, "psf_method2")) != PSF_OK) return st;
  if ((st = validate_grid(N, cell)) != PSF_OK) return st;
  if (S == nullptr) return fail(PSF_EINVAL, "S is NULL");
  const psf_src g = effective_grid(N, cell);
  const PatchPlan plan = plan_patch(obs, &g, prec, kTargetWorkgroups);
  const SpectrumLayout L = spectrum_layout(obs, plan, N);
  if (ws == nullptr || ws_bytes < L.total)
    return fail(PSF_EWORKSPACE, "psf_method2_spectrum needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  if ((st = check_device()) != PSF_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* w = static_cast<uint8_t*>(ws);
  BinRec* rec = reinterpret_cast<BinRec*>(w);
  float2* c = reinterpret_cast<float2*>(w + align_up(static_cast<size_t>(obs->K) * sizeof(BinRec), 256));
  float* partial = reinterpret_cast<float*>(reinterpret_cast<uint8_t*>(c) +
                                            align_up(static_cast<size_t>(obs->K) * sizeof(float2), 256));
  float* Peff = reinterpret_cast<float*>(w + L.Peff);
  hipError_t e;
  if (obs->K > 0) {
    // At the phase centre every sample's phase difference is exactly 0, so
    // D_k = 1 and u' = u: the effective PSF.
    e = launch_decorr(view(obs), 0.0, 0.0, cell, cell, nullptr, nullptr, rec, c, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "k_decorr launch");
  }
  if ((st = contract(obs, &g, plan, prec, rec, c, partial, Peff, s)) != PSF_OK) return st;
  const int64_t NN = static_cast<int64_t>(N) * N;
  float2* Sc = reinterpret_cast<float2*>(S);
  hipLaunchKernelGGL(k_m2_load, dim3(static_cast<unsigned>((NN + 255) / 256)), dim3(256), 0, s, Peff, g.nm, Sc, N);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_m2_load launch");
  return fft2(Sc, N, 1, -1.0f, s);
}

int psf_method2_patch(int32_t N, double cell, const float* S, int32_t n_src, const double* h_dirs, double dt_bin,
                      double dnu_bin, double nu, float* P, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  int st;
  if ((st = validate_grid(N, cell)) != PSF_OK) return st;
  if (S == nullptr || P == nullptr) return fail(PSF_EINVAL, "S or P is NULL");
  if (n_src < 1 || h_dirs == nullptr) return fail(PSF_EINVAL, "need n_src >= 1 directions");
  if (!(dt_bin >= 0.0) || !(dnu_bin >= 0.0) || !(nu > 0.0) || !std::isfinite(dt_bin) || !std::isfinite(dnu_bin) ||
      !std::isfinite(nu))
    return fail(PSF_EINVAL, "bin duration, bandwidth and frequency must be finite, >= 0 (nu > 0)");
  for (int q = 0; q < n_src; ++q) {
    const double l0 = h_dirs[2 * q], m0 = h_dirs[2 * q + 1];
    if (!std::isfinite(l0) || !std::isfinite(m0) || l0 * l0 + m0 * m0 >= 1.0)
      return fail(PSF_EINVAL, "direction %d outside the sky", q);
  }
  const size_t need = patch_m2_workspace(N, n_src);
  if (ws == nullptr || ws_bytes < need)
    return fail(PSF_EWORKSPACE, "psf_method2_patch needs %zu workspace bytes, got %zu", need, ws_bytes);
  if ((st = check_device()) != PSF_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  float2* work = static_cast<float2*>(ws);
  const int64_t NN = static_cast<int64_t>(N) * N;
  const unsigned nb = static_cast<unsigned>((NN + 255) / 256);
  const double du = 1.0 / (N * cell);
  for (int q0 = 0; q0 < n_src; q0 += kChunk) {
    const int nq = std::min(kChunk, n_src - q0);
    Dirs d{};
    for (int q = 0; q < nq; ++q) {
      d.l0[q] = h_dirs[2 * (q0 + q)];
      d.m0[q] = h_dirs[2 * (q0 + q) + 1];
    }
    hipLaunchKernelGGL(k_m2_dhat, dim3(nb, nq), dim3(256), 0, s, reinterpret_cast<const float2*>(S), work, N, du,
                       dt_bin, dnu_bin / nu, d, static_cast<const double*>(nullptr));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_m2_dhat launch");
    if ((st = fft2(work, N, nq, 1.0f, s)) != PSF_OK) return st;
    hipLaunchKernelGGL(k_m2_store, dim3(nb, nq), dim3(256), 0, s, work, P + q0 * NN, N,
                       static_cast<float>(1.0 / static_cast<double>(NN)));
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_m2_store launch");
  }
  return PSF_OK;
}

}  // extern "C"
