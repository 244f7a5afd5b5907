// Deconvolution with position-dependent PSFs [Algorithm 2, Hogbom CLEAN]:
// every minor cycle finds the peak of |residual|, computes the distorted PSF
// at that direction on the image grid (the same decorrelation, phase-factor
// and contraction kernels as psf_patch), and subtracts gain * peak times the
// PSF normalised to 1 at the peak.  The peak search and the subtraction are
// kernels.  psf_clean_hogbom reads back the peak (one synchronisation per
// cycle) to place the next PSF and to stop at the threshold;
// psf_clean_hogbom_device places it on the device (the direction goes to a
// device source record that the decorrelation and the contraction read at
// run time) and runs a fixed number of cycles, so that it can be captured.
#include <algorithm>
#include <cmath>

#include "psf_host.hpp"

namespace psf {

namespace {

constexpr int kMaxThreads = 256;
constexpr int kMaxBlocks = 512;

struct Peak {
  float absval;
  float val;
  int64_t idx;
};

// Larger |value| wins; equal |value|: the smaller index (the first maximum
// in row-major order).
__device__ __forceinline__ Peak better(const Peak& a, const Peak& b) {
  if (a.absval > b.absval) return a;
  if (b.absval > a.absval) return b;
  return a.idx <= b.idx ? a : b;
}

__device__ Peak block_best(Peak p) {
  __shared__ float s_abs[kMaxThreads / 64], s_val[kMaxThreads / 64];
  __shared__ int64_t s_idx[kMaxThreads / 64];
  for (int o = 32; o > 0; o >>= 1) {
    Peak q;
    q.absval = __shfl_xor(p.absval, o);
    q.val = __shfl_xor(p.val, o);
    q.idx = __shfl_xor(p.idx, o);
    p = better(p, q);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    s_abs[wave] = p.absval;
    s_val[wave] = p.val;
    s_idx[wave] = p.idx;
  }
  __syncthreads();
  Peak r{-1.0f, 0.0f, INT64_MAX};
  for (int w = 0; w < kMaxThreads / 64; ++w) r = better(r, Peak{s_abs[w], s_val[w], s_idx[w]});
  return r;
}

// Per-block best of a grid-strided range; one entry per block.
__global__ __launch_bounds__(kMaxThreads) void k_absmax_partial(const float* __restrict__ x, int64_t n,
                                                                 Peak* __restrict__ part) {
  Peak p{-1.0f, 0.0f, INT64_MAX};
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kMaxThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kMaxThreads)
    p = better(p, Peak{fabsf(x[i]), x[i], i});
  const Peak r = block_best(p);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ __launch_bounds__(kMaxThreads) void k_absmax_final(const Peak* __restrict__ part, int nb,
                                                               Peak* __restrict__ out) {
  Peak p{-1.0f, 0.0f, INT64_MAX};
  for (int i = threadIdx.x; i < nb; i += kMaxThreads) p = better(p, part[i]);
  const Peak r = block_best(p);
  if (threadIdx.x == 0) *out = r;
}

// residual -= gain * peak * P / P[peak index]
__global__ __launch_bounds__(kMaxThreads) void k_clean_subtract(float* __restrict__ res, const float* __restrict__ P,
                                                                 int64_t n, const Peak* __restrict__ pk, float gain) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kMaxThreads + threadIdx.x;
  if (i >= n) return;
  const float p0 = P[pk->idx];
  const float scale = p0 != 0.0f ? gain * pk->val / p0 : 0.0f;  // a zero PSF subtracts nothing
  res[i] -= scale * P[i];
}

// residual -= gain * peak * P / P(centre), P a centred N x N PSF laid with
// its centre on pixel (pi, pj); pixels beyond its extent are not changed.
__global__ __launch_bounds__(kMaxThreads) void k_clean_subtract_laid(float* __restrict__ res, int nl, int nm,
                                                                      const float* __restrict__ P, int N, int pi,
                                                                      int pj, const Peak* __restrict__ pk,
                                                                      float gain) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kMaxThreads + threadIdx.x;
  if (idx >= static_cast<int64_t>(nl) * nm) return;
  const int a = static_cast<int>(idx / nm), b = static_cast<int>(idx - static_cast<int64_t>(a) * nm);
  const int u = a - pi + N / 2, v = b - pj + N / 2;
  if (u < 0 || u >= N || v < 0 || v >= N) return;
  const float scale = gain * pk->val / P[static_cast<int64_t>(N / 2) * N + N / 2];
  res[idx] -= scale * P[static_cast<int64_t>(u) * N + v];
}

// The device-side state of psf_clean_hogbom_device: the source record the
// PSF kernels read (psf_src layout: l0, m0, l_first, m_first, dl, dm, ...),
// whether cleaning goes on, and the current cycle's amplitude.
struct CleanState {
  psf_src src;
  float amp;
  int32_t active;
  int32_t pi, pj;  // the current peak pixel (where a Method-2 PSF is laid)
};

__global__ void k_clean_init(CleanState* __restrict__ st, psf_src grid, int32_t* __restrict__ n_comp) {
  // the grid's centre pixel: a valid direction for cycles that subtract nothing
  grid.l0 = grid.l_first + (grid.nl / 2) * grid.dl;
  grid.m0 = grid.m_first + (grid.nm / 2) * grid.dm;
  st->src = grid;
  st->amp = 0.0f;
  st->active = 1;
  st->pi = grid.nl / 2;
  st->pj = grid.nm / 2;
  *n_comp = 0;
}

// Cycle `it`: the peak's pixel becomes the PSF's direction and component
// `it`, unless cleaning has stopped (|peak| below the threshold or zero, or
// a direction off the sky), after which every cycle subtracts nothing.
__global__ void k_clean_place(CleanState* __restrict__ st, const Peak* __restrict__ pk, int64_t n, int nm,
                              double threshold, double gain, int it, int32_t* __restrict__ ci,
                              int32_t* __restrict__ cj, float* __restrict__ ca, int32_t* __restrict__ n_comp) {
  // the direction rounded as the host forms it in psf_clean_hogbom (no fused multiply-add)
#pragma clang fp contract(off)
  const Peak p = *pk;
  bool go = st->active != 0 && p.idx >= 0 && p.idx < n && p.absval >= threshold && p.absval != 0.0f;
  int i = 0, j = 0;
  double l0 = 0.0, m0 = 0.0;
  if (go) {
    i = static_cast<int>(p.idx / nm);
    j = static_cast<int>(p.idx % nm);
    l0 = st->src.l_first + i * st->src.dl;
    m0 = st->src.m_first + j * st->src.dm;
    go = l0 * l0 + m0 * m0 < 1.0;
  }
  if (!go) {
    st->active = 0;
    st->amp = 0.0f;
    return;
  }
  st->src.l0 = l0;
  st->src.m0 = m0;
  st->pi = i;
  st->pj = j;
  st->amp = static_cast<float>(gain) * p.val;
  ci[it] = i;
  cj[it] = j;
  ca[it] = static_cast<float>(gain * p.val);
  *n_comp = it + 1;
}

// residual -= amp * P / P[peak index] (amp = gain * peak, or 0 once
// cleaning has stopped), as k_clean_subtract.
__global__ __launch_bounds__(kMaxThreads) void k_clean_subtract_dev(float* __restrict__ res,
                                                                     const float* __restrict__ P, int64_t n,
                                                                     const Peak* __restrict__ pk,
                                                                     const CleanState* __restrict__ st) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kMaxThreads + threadIdx.x;
  if (i >= n || st->active == 0) return;
  const float p0 = P[pk->idx];
  const float scale = p0 != 0.0f ? st->amp / p0 : 0.0f;
  res[i] -= scale * P[i];
}

// residual -= amp * P / P(centre) with the Method-2 PSF laid on the
// current peak pixel (both from the device state), as k_clean_subtract_laid.
__global__ __launch_bounds__(kMaxThreads) void k_clean_subtract_laid_dev(float* __restrict__ res, int nl, int nm,
                                                                          const float* __restrict__ P, int N,
                                                                          const CleanState* __restrict__ st) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kMaxThreads + threadIdx.x;
  if (idx >= static_cast<int64_t>(nl) * nm || st->active == 0) return;
  const int a = static_cast<int>(idx / nm), b = static_cast<int>(idx - static_cast<int64_t>(a) * nm);
  const int u = a - st->pi + N / 2, v = b - st->pj + N / 2;
  if (u < 0 || u >= N || v < 0 || v >= N) return;
  const float scale = st->amp / P[static_cast<int64_t>(N / 2) * N + N / 2];
  res[idx] -= scale * P[static_cast<int64_t>(u) * N + v];
}

struct M2CleanLayout {
  size_t part, peak, P, work, state, total;
};

M2CleanLayout m2_clean_layout(int32_t N) {
  M2CleanLayout L;
  L.part = 0;
  L.peak = align_up(kMaxBlocks * sizeof(Peak), 256);
  L.P = L.peak + align_up(sizeof(Peak), 256);
  L.work = L.P + align_up(static_cast<size_t>(N) * N * sizeof(float), 256);
  L.state = L.work + align_up(static_cast<size_t>(N) * N * sizeof(float2), 256);
  L.total = L.state + align_up(sizeof(CleanState), 256);
  return L;
}

int validate_m2_clean(int32_t N, const psf_src* grid) {
  int st;
  if ((st = validate_src(grid, 0)) != PSF_OK) return st;
  if (N < 16 || N > 4096 || (N & (N - 1)) != 0) return fail(PSF_EINVAL, "N=%d must be a power of two in 16..4096", N);
  if (!(std::fabs(grid->dl - grid->dm) <= 1e-12 * std::fabs(grid->dl)))
    return fail(PSF_EINVAL, "Method-2 CLEAN needs square cells (dl = dm)");
  return PSF_OK;
}

struct CleanLayout {
  size_t patch, P, part, peak, state, total;
};

CleanLayout clean_layout(const psf_obs* o, const psf_src* grid, int prec) {
  CleanLayout L;
  const PatchPlan plan = plan_patch(o, grid, prec, kTargetWorkgroups);
  L.patch = 0;
  L.P = align_up(patch_workspace(o, plan), 256);
  L.part = L.P + align_up(static_cast<size_t>(grid->nl) * grid->nm * sizeof(float), 256);
  L.peak = L.part + align_up(kMaxBlocks * sizeof(Peak), 256);
  L.state = L.peak + align_up(sizeof(Peak), 256);
  L.total = L.state + align_up(sizeof(CleanState), 256);
  return L;
}

int validate_clean(const psf_obs* obs, const psf_src* grid, int prec) {
  int st;
  if ((st = validate_obs(obs)) != PSF_OK) return st;
  if ((st = validate_prec(prec)) != PSF_OK) return st;
  if ((st = reject_normalise(prec, "psf_clean_hogbom")) != PSF_OK) return st;
  if ((st = validate_src(grid, 0)) != PSF_OK) return st;
  return PSF_OK;
}

}  // namespace

}  // namespace psf

using namespace psf;

extern "C" {

int psf_clean_workspace_bytes(const psf_obs* obs, const psf_src* h_grid, int prec, size_t* out) {
  clear_error();
  int st;
  if ((st = validate_clean(obs, h_grid, prec)) != PSF_OK) return st;
  if (out == nullptr) return fail(PSF_EINVAL, "out is NULL");
  *out = clean_layout(obs, h_grid, prec).total;
  return PSF_OK;
}

int psf_clean_hogbom(const psf_obs* obs, const psf_src* h_grid, float* residual, int32_t max_iter, double gain,
                     double threshold, int prec, int32_t* comp_i, int32_t* comp_j, float* comp_amp,
                     int32_t* n_comp, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  int st;
  if ((st = validate_clean(obs, h_grid, prec)) != PSF_OK) return st;
  if (residual == nullptr || n_comp == nullptr) return fail(PSF_EINVAL, "residual or n_comp is NULL");
  if (max_iter < 0) return fail(PSF_EINVAL, "max_iter < 0");
  if (max_iter > 0 && (comp_i == nullptr || comp_j == nullptr || comp_amp == nullptr))
    return fail(PSF_EINVAL, "component arrays are NULL");
  if (!(gain > 0.0 && gain <= 1.0)) return fail(PSF_EINVAL, "gain %g outside (0, 1]", gain);
  if (!(threshold >= 0.0)) return fail(PSF_EINVAL, "threshold must be >= 0");
  const CleanLayout L = clean_layout(obs, h_grid, prec);
  if (ws == nullptr || ws_bytes < L.total)
    return fail(PSF_EWORKSPACE, "psf_clean_hogbom needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  if ((st = check_device()) != PSF_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* w = static_cast<uint8_t*>(ws);
  BinRec* rec = reinterpret_cast<BinRec*>(w);
  float2* c = reinterpret_cast<float2*>(w + align_up(static_cast<size_t>(obs->K) * sizeof(BinRec), 256));
  float* partial = reinterpret_cast<float*>(reinterpret_cast<uint8_t*>(c) +
                                            align_up(static_cast<size_t>(obs->K) * sizeof(float2), 256));
  float* P = reinterpret_cast<float*>(w + L.P);
  Peak* part = reinterpret_cast<Peak*>(w + L.part);
  Peak* peak = reinterpret_cast<Peak*>(w + L.peak);
  const PatchPlan plan = plan_patch(obs, h_grid, prec, kTargetWorkgroups);
  const int64_t n = static_cast<int64_t>(h_grid->nl) * h_grid->nm;
  const int nb = static_cast<int>(std::min<int64_t>(kMaxBlocks, (n + kMaxThreads - 1) / kMaxThreads));
  *n_comp = 0;
  if (obs->K == 0) return PSF_OK;  // no visibilities: the PSF is zero, nothing to subtract
  for (int it = 0; it < max_iter; ++it) {
    hipLaunchKernelGGL(k_absmax_partial, dim3(nb), dim3(kMaxThreads), 0, s, residual, n, part);
    hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(kMaxThreads), 0, s, part, nb, peak);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "peak search launch");
    Peak hp;
    if ((e = hipMemcpyAsync(&hp, peak, sizeof(Peak), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return hip_fail(e, "peak read-back");
    if (hp.idx < 0 || hp.idx >= n || !(hp.absval >= threshold) || hp.absval == 0.0f) break;
    const int i = static_cast<int>(hp.idx / h_grid->nm), j = static_cast<int>(hp.idx % h_grid->nm);
    psf_src src = *h_grid;
    src.l0 = h_grid->l_first + i * h_grid->dl;
    src.m0 = h_grid->m_first + j * h_grid->dm;
    if (src.l0 * src.l0 + src.m0 * src.m0 >= 1.0) return fail(PSF_EINVAL, "peak pixel outside the sky");
    if (obs->K > 0 &&
        (e = launch_decorr(view(obs), src.l0, src.m0, src.dl, src.dm, nullptr, nullptr, rec, c, nullptr, s)) !=
            hipSuccess)
      return hip_fail(e, "k_decorr launch");
    if ((st = contract(obs, &src, plan, prec, rec, c, partial, P, s)) != PSF_OK) return st;
    hipLaunchKernelGGL(k_clean_subtract, dim3(static_cast<unsigned>((n + kMaxThreads - 1) / kMaxThreads)),
                       dim3(kMaxThreads), 0, s, residual, P, n, peak, static_cast<float>(gain));
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_clean_subtract launch");
    comp_i[it] = i;
    comp_j[it] = j;
    comp_amp[it] = static_cast<float>(gain * hp.val);
    *n_comp = it + 1;
  }
  hipError_t e = hipStreamSynchronize(s);
  return e == hipSuccess ? PSF_OK : hip_fail(e, "hipStreamSynchronize");
}

int psf_clean_hogbom_device(const psf_obs* obs, const psf_src* h_grid, float* residual, int32_t n_iter, double gain,
                            double threshold, int prec, int32_t* comp_i, int32_t* comp_j, float* comp_amp,
                            int32_t* n_comp, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  int st;
  if ((st = validate_clean(obs, h_grid, prec)) != PSF_OK) return st;
  if (residual == nullptr || n_comp == nullptr) return fail(PSF_EINVAL, "residual or n_comp is NULL");
  if (n_iter < 0) return fail(PSF_EINVAL, "n_iter < 0");
  if (n_iter > 0 && (comp_i == nullptr || comp_j == nullptr || comp_amp == nullptr))
    return fail(PSF_EINVAL, "component arrays are NULL");
  if (!(gain > 0.0 && gain <= 1.0)) return fail(PSF_EINVAL, "gain %g outside (0, 1]", gain);
  if (!(threshold >= 0.0)) return fail(PSF_EINVAL, "threshold must be >= 0");
  const CleanLayout L = clean_layout(obs, h_grid, prec);
  if (ws == nullptr || ws_bytes < L.total)
    return fail(PSF_EWORKSPACE, "psf_clean_hogbom_device needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  if ((st = check_device()) != PSF_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* w = static_cast<uint8_t*>(ws);
  BinRec* rec = reinterpret_cast<BinRec*>(w);
  float2* c = reinterpret_cast<float2*>(w + align_up(static_cast<size_t>(obs->K) * sizeof(BinRec), 256));
  float* partial = reinterpret_cast<float*>(reinterpret_cast<uint8_t*>(c) +
                                            align_up(static_cast<size_t>(obs->K) * sizeof(float2), 256));
  float* P = reinterpret_cast<float*>(w + L.P);
  Peak* part = reinterpret_cast<Peak*>(w + L.part);
  Peak* peak = reinterpret_cast<Peak*>(w + L.peak);
  CleanState* state = reinterpret_cast<CleanState*>(w + L.state);
  const double* dir = reinterpret_cast<const double*>(&state->src);
  const PatchPlan plan = plan_patch(obs, h_grid, prec, kTargetWorkgroups);
  const int64_t n = static_cast<int64_t>(h_grid->nl) * h_grid->nm;
  const int nb = static_cast<int>(std::min<int64_t>(kMaxBlocks, (n + kMaxThreads - 1) / kMaxThreads));
  hipLaunchKernelGGL(k_clean_init, dim3(1), dim3(1), 0, s, state, *h_grid, n_comp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_clean_init launch");
  if (obs->K == 0) return PSF_OK;  // no visibilities: the PSF is zero, nothing to subtract
  for (int it = 0; it < n_iter; ++it) {
    hipLaunchKernelGGL(k_absmax_partial, dim3(nb), dim3(kMaxThreads), 0, s, residual, n, part);
    hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(kMaxThreads), 0, s, part, nb, peak);
    hipLaunchKernelGGL(k_clean_place, dim3(1), dim3(1), 0, s, state, peak, n, h_grid->nm, threshold, gain, it,
                       comp_i, comp_j, comp_amp, n_comp);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "peak search launch");
    if ((e = launch_decorr(view(obs), 0.0, 0.0, h_grid->dl, h_grid->dm, nullptr, nullptr, rec, c, nullptr, s,
                           dir)) != hipSuccess)
      return hip_fail(e, "k_decorr launch");
    if ((st = contract(obs, h_grid, plan, prec, rec, c, partial, P, s, dir)) != PSF_OK) return st;
    hipLaunchKernelGGL(k_clean_subtract_dev, dim3(static_cast<unsigned>((n + kMaxThreads - 1) / kMaxThreads)),
                       dim3(kMaxThreads), 0, s, residual, P, n, peak, state);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_clean_subtract_dev launch");
  }
  return PSF_OK;
}

int psf_clean_method2_workspace_bytes(int32_t N, const psf_src* h_grid, size_t* out) {
  clear_error();
  int st;
  if ((st = validate_m2_clean(N, h_grid)) != PSF_OK) return st;
  if (out == nullptr) return fail(PSF_EINVAL, "out is NULL");
  *out = m2_clean_layout(N).total;
  return PSF_OK;
}

int psf_clean_hogbom_method2(int32_t N, const float* S, const psf_src* h_grid, float* residual, int32_t max_iter,
                             double gain, double threshold, double dt_bin, double dnu_bin, double nu,
                             int32_t* comp_i, int32_t* comp_j, float* comp_amp, int32_t* n_comp, void* ws,
                             size_t ws_bytes, void* stream) {
  clear_error();
  int st;
  if ((st = validate_m2_clean(N, h_grid)) != PSF_OK) return st;
  if (S == nullptr || residual == nullptr || n_comp == nullptr) return fail(PSF_EINVAL, "S, residual or n_comp is NULL");
  if (max_iter < 0) return fail(PSF_EINVAL, "max_iter < 0");
  if (max_iter > 0 && (comp_i == nullptr || comp_j == nullptr || comp_amp == nullptr))
    return fail(PSF_EINVAL, "component arrays are NULL");
  if (!(gain > 0.0 && gain <= 1.0)) return fail(PSF_EINVAL, "gain %g outside (0, 1]", gain);
  if (!(threshold >= 0.0)) return fail(PSF_EINVAL, "threshold must be >= 0");
  const M2CleanLayout L = m2_clean_layout(N);
  if (ws == nullptr || ws_bytes < L.total)
    return fail(PSF_EWORKSPACE, "psf_clean_hogbom_method2 needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  if ((st = check_device()) != PSF_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* w = static_cast<uint8_t*>(ws);
  Peak* part = reinterpret_cast<Peak*>(w + L.part);
  Peak* peak = reinterpret_cast<Peak*>(w + L.peak);
  float* P = reinterpret_cast<float*>(w + L.P);
  void* work = w + L.work;
  const size_t work_bytes = L.total - L.work;
  const int64_t n = static_cast<int64_t>(h_grid->nl) * h_grid->nm;
  const int nb = static_cast<int>(std::min<int64_t>(kMaxBlocks, (n + kMaxThreads - 1) / kMaxThreads));
  *n_comp = 0;
  for (int it = 0; it < max_iter; ++it) {
    hipLaunchKernelGGL(k_absmax_partial, dim3(nb), dim3(kMaxThreads), 0, s, residual, n, part);
    hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(kMaxThreads), 0, s, part, nb, peak);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "peak search launch");
    Peak hp;
    if ((e = hipMemcpyAsync(&hp, peak, sizeof(Peak), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return hip_fail(e, "peak read-back");
    if (hp.idx < 0 || hp.idx >= n || !(hp.absval >= threshold) || hp.absval == 0.0f) break;
    const int i = static_cast<int>(hp.idx / h_grid->nm), j = static_cast<int>(hp.idx % h_grid->nm);
    const double dir[2] = {h_grid->l_first + i * h_grid->dl, h_grid->m_first + j * h_grid->dm};
    if ((st = psf_method2_patch(N, h_grid->dl, S, 1, dir, dt_bin, dnu_bin, nu, P, work, work_bytes, stream)) !=
        PSF_OK)
      return st;
    hipLaunchKernelGGL(k_clean_subtract_laid, dim3(static_cast<unsigned>((n + kMaxThreads - 1) / kMaxThreads)),
                       dim3(kMaxThreads), 0, s, residual, h_grid->nl, h_grid->nm, P, N, i, j, peak,
                       static_cast<float>(gain));
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_clean_subtract_laid launch");
    comp_i[it] = i;
    comp_j[it] = j;
    comp_amp[it] = static_cast<float>(gain * hp.val);
    *n_comp = it + 1;
  }
  hipError_t e = hipStreamSynchronize(s);
  return e == hipSuccess ? PSF_OK : hip_fail(e, "hipStreamSynchronize");
}

int psf_clean_hogbom_method2_device(int32_t N, const float* S, const psf_src* h_grid, float* residual,
                                    int32_t n_iter, double gain, double threshold, double dt_bin, double dnu_bin,
                                    double nu, int32_t* comp_i, int32_t* comp_j, float* comp_amp, int32_t* n_comp,
                                    void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  int st;
  if ((st = validate_m2_clean(N, h_grid)) != PSF_OK) return st;
  if (S == nullptr || residual == nullptr || n_comp == nullptr) return fail(PSF_EINVAL, "S, residual or n_comp is NULL");
  if (n_iter < 0) return fail(PSF_EINVAL, "n_iter < 0");
  if (n_iter > 0 && (comp_i == nullptr || comp_j == nullptr || comp_amp == nullptr))
    return fail(PSF_EINVAL, "component arrays are NULL");
  if (!(gain > 0.0 && gain <= 1.0)) return fail(PSF_EINVAL, "gain %g outside (0, 1]", gain);
  if (!(threshold >= 0.0)) return fail(PSF_EINVAL, "threshold must be >= 0");
  if (!(dt_bin >= 0.0) || !(dnu_bin >= 0.0) || !(nu > 0.0) || !std::isfinite(dt_bin) || !std::isfinite(dnu_bin) ||
      !std::isfinite(nu))
    return fail(PSF_EINVAL, "bin duration, bandwidth and frequency must be finite, >= 0 (nu > 0)");
  const M2CleanLayout L = m2_clean_layout(N);
  if (ws == nullptr || ws_bytes < L.total)
    return fail(PSF_EWORKSPACE, "psf_clean_hogbom_method2_device needs %zu workspace bytes, got %zu", L.total,
                ws_bytes);
  if ((st = check_device()) != PSF_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* w = static_cast<uint8_t*>(ws);
  Peak* part = reinterpret_cast<Peak*>(w + L.part);
  Peak* peak = reinterpret_cast<Peak*>(w + L.peak);
  float* P = reinterpret_cast<float*>(w + L.P);
  float2* work = reinterpret_cast<float2*>(w + L.work);
  CleanState* state = reinterpret_cast<CleanState*>(w + L.state);
  const double* dir = reinterpret_cast<const double*>(&state->src);
  const int64_t n = static_cast<int64_t>(h_grid->nl) * h_grid->nm;
  const int nb = static_cast<int>(std::min<int64_t>(kMaxBlocks, (n + kMaxThreads - 1) / kMaxThreads));
  hipLaunchKernelGGL(k_clean_init, dim3(1), dim3(1), 0, s, state, *h_grid, n_comp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_clean_init launch");
  for (int it = 0; it < n_iter; ++it) {
    hipLaunchKernelGGL(k_absmax_partial, dim3(nb), dim3(kMaxThreads), 0, s, residual, n, part);
    hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(kMaxThreads), 0, s, part, nb, peak);
    hipLaunchKernelGGL(k_clean_place, dim3(1), dim3(1), 0, s, state, peak, n, h_grid->nm, threshold, gain, it,
                       comp_i, comp_j, comp_amp, n_comp);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "peak search launch");
    if ((st = method2_patch_device_dir(N, h_grid->dl, S, dir, dt_bin, dnu_bin, nu, P, work, s)) != PSF_OK) return st;
    hipLaunchKernelGGL(k_clean_subtract_laid_dev, dim3(static_cast<unsigned>((n + kMaxThreads - 1) / kMaxThreads)),
                       dim3(kMaxThreads), 0, s, residual, h_grid->nl, h_grid->nm, P, N, state);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_clean_subtract_laid_dev launch");
  }
  return PSF_OK;
}

}  // extern "C"
