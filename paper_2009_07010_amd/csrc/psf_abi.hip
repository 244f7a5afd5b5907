// Host side of libpsfdecorr: argument validation, workspace planning, launch
// sequencing and error reporting behind the C ABI declared in include/psf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/psf.h"
#include "psf_host.hpp"
#include "psf_kernels.hpp"

namespace psf {

// ------------------------------------------------------------------ errors
static thread_local char g_msg[512] = "";

void clear_error() { g_msg[0] = 0; }

int fail(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof g_msg, fmt, ap);
  va_end(ap);
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(PSF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------------------ device
int check_device() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  static std::mutex mu;
  static std::vector<int> state;  // per device: 0 unknown, 1 ok, 2 unsupported
  std::lock_guard<std::mutex> lock(mu);
  if (static_cast<int>(state.size()) <= dev) state.resize(dev + 1, 0);
  if (state[dev] == 0) {
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    state[dev] = std::strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
  }
  if (state[dev] != 1) return fail(PSF_EUNSUPPORTED, "device %d is not gfx950 (MI355X)", dev);
  return PSF_OK;
}

// ------------------------------------------------------------------ validation
int validate_obs(const psf_obs* o) {
  if (o == nullptr) return fail(PSF_EINVAL, "obs is NULL");
  if (o->reserved != 0) return fail(PSF_EINVAL, "obs.reserved must be 0");
  if (o->n_bl < 0 || o->n_t < 1 || o->n_ch < 1)
    return fail(PSF_EINVAL, "bad sizes n_bl=%d n_t=%d n_ch=%d", o->n_bl, o->n_t, o->n_ch);
  if (o->K < 0 || o->n_tb < 0) return fail(PSF_EINVAL, "negative K or n_tb");
  if (o->n_bl == 0 && (o->K != 0 || o->n_tb != 0)) return fail(PSF_EINVAL, "no baselines but K != 0");
  if (o->n_bl > 0 && o->K < o->n_bl) return fail(PSF_EINVAL, "K=%lld smaller than n_bl=%d", (long long)o->K, o->n_bl);
  if (o->n_bl > 0 && (static_cast<int64_t>(o->n_bl) * o->n_t * o->n_ch) < o->K)
    return fail(PSF_EINVAL, "K exceeds the number of samples");
  if (o->K > (int64_t(1) << 40)) return fail(PSF_EINVAL, "K too large");
  if (o->n_bl > 0) {
    if (!o->uvw_m || !o->freq_hz || !o->bl_bin || !o->bl_koff || !o->bl_tboff || !o->uvw_c_m || !o->W)
      return fail(PSF_EINVAL, "an observation array pointer is NULL");
  }
  return PSF_OK;
}

int validate_src(const psf_src* s, int idx) {
  if (s == nullptr) return fail(PSF_EINVAL, "source %d is NULL", idx);
  if (s->nl < 1 || s->nm < 1 || s->nl > 4096 || s->nm > 4096)
    return fail(PSF_EINVAL, "source %d: patch %dx%d outside 1..4096", idx, s->nl, s->nm);
  const double v[6] = {s->l0, s->m0, s->l_first, s->m_first, s->dl, s->dm};
  for (double x : v)
    if (!std::isfinite(x)) return fail(PSF_EINVAL, "source %d: non-finite direction or grid", idx);
  if (s->l0 * s->l0 + s->m0 * s->m0 >= 1.0) return fail(PSF_EINVAL, "source %d: l0^2 + m0^2 >= 1", idx);
  if (s->out_off < 0) return fail(PSF_EINVAL, "source %d: negative out_off", idx);
  return PSF_OK;
}

int validate_prec(int prec) {
  const int base = prec_base(prec);
  if (base < PSF_FP32 || base > PSF_SR_FP16) return fail(PSF_EINVAL, "unknown precision %d", prec);
  return PSF_OK;
}

int reject_normalise(int prec, const char* entry) {
  if (prec_normalise(prec)) return fail(PSF_EINVAL, "%s does not take PSF_NORMALISE", entry);
  return PSF_OK;
}

ObsView view(const psf_obs* o) {
  ObsView v;
  v.uvw = o->uvw_m;
  v.freq = o->freq_hz;
  v.bl_bin = o->bl_bin;
  v.koff = o->bl_koff;
  v.tboff = o->bl_tboff;
  v.uvw_c = o->uvw_c_m;
  v.W = o->W;
  v.win_t = o->win_t;
  v.win_c = o->win_c;
  v.K = o->K;
  v.n_tb = o->n_tb;
  v.n_bl = o->n_bl;
  v.n_t = o->n_t;
  v.n_ch = o->n_ch;
  return v;
}

// ------------------------------------------------------------------ planning
size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool sym_source(const psf_src* s) { return sym_patch_size(s->nl, s->nm); }

// Cost of one chunk (16 visibilities, 32 in the symmetric form) of each tile
// type of a tile plan, in SIMD cycles on MI355X: matrix-core time of the
// busiest SIMD's two waves plus the vector time of its phase-factor rows
// (one A-row and one B-row wave, about 10 instructions per row and 100 per
// chunk for seeds and records, twice that in the symmetric form, 4.7 cycles
// each).  Measured kernels behave closer to the sum of the two than to their
// maximum.
static void chunk_costs(const TilePlan& t, int prec, bool sym, int64_t K, double cost[2][2]) {
  // (the mixed and stochastic forms run two and one products where they run
  // at all, see contraction_prec: plans of their split-FP16 routes are
  // split-FP16 plans)
  const bool many = sym && K >= kMixedMinK;
  const double mfma_per_block = prec == PSF_FP32                     ? 256.0
                                : prec == PSF_PLAIN_BF16             ? 16.0
                                : prec == PSF_MIXED_FP16 && many ? 32.0
                                : prec == PSF_SR_FP16 && many    ? 16.0
                                                                     : 48.0;
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      const double mf = mfma_per_block * tile_max_simd_blocks(t.tbi[r], t.tbj[c], sym);
      const double gen = 4.7 * (10.0 * (t.tbi[r] + t.tbj[c]) + (sym ? 200.0 : 100.0));
      cost[r][c] = mf + gen;
    }
}

static int64_t chunk_count(const psf_obs* o, bool sym) {
  const int64_t ch = sym ? kPatchChunkSym : kPatchChunk;
  return std::max<int64_t>(1, (o->K + ch - 1) / ch);
}

double patch_work(const psf_obs* o, const psf_src* s, int prec) {
  TilePlan t;
  plan_tiles((s->nl + 15) / 16, (s->nm + 15) / 16, &t);
  const bool sym = sym_source(s);
  double cost[2][2];
  chunk_costs(t, prec, sym, o->K, cost);
  const int cnt_i[2] = {t.ti_a, t.ti_b}, cnt_j[2] = {t.tj_a, t.tj_b};
  const double chunks = static_cast<double>(chunk_count(o, sym));
  double work = 0.0;
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) work += static_cast<double>(cnt_i[r]) * cnt_j[c] * cost[r][c] * chunks;
  return work;
}

PatchPlan plan_patch_items(const psf_obs* o, const psf_src* s, int prec, double item_work) {
  PatchPlan p;
  TilePlan& t = p.tp;
  plan_tiles((s->nl + 15) / 16, (s->nm + 15) / 16, &t);
  p.sym = sym_source(s);
  const int64_t chunks = chunk_count(o, p.sym);
  const int64_t ch = p.sym ? kPatchChunkSym : kPatchChunk;
  double cost[2][2];
  chunk_costs(t, prec, p.sym, o->K, cost);
  // k-slices per tile so that every work item costs about item_work
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      int64_t n = static_cast<int64_t>(std::llround(cost[r][c] * static_cast<double>(chunks) / item_work));
      n = std::min<int64_t>(std::max<int64_t>(1, n), chunks);
      t.ns[r][c] = static_cast<int>(n);
      t.kps[r][c] = ((chunks + n - 1) / n) * ch;
    }
  p.partial_elems = tile_plan_partial_elems(t);
  return p;
}

PatchPlan plan_patch(const psf_obs* o, const psf_src* s, int prec, int target_wgs) {
  TilePlan t;
  plan_tiles((s->nl + 15) / 16, (s->nm + 15) / 16, &t);
  const int wgs = tile_wgs_per_cu(t, launch_prec(prec, o->K, sym_source(s)));
  return plan_patch_items(o, s, prec, patch_work(o, s, prec) / (target_wgs * wgs));
}

size_t patch_workspace(const psf_obs* o, const PatchPlan& p) {
  size_t b = 0;
  b += align_up(static_cast<size_t>(o->K) * sizeof(BinRec), 256);  // (u', v')
  b += align_up(static_cast<size_t>(o->K) * sizeof(float2), 256);   // c = W D
  b += align_up(p.partial_elems * sizeof(float), 256);
  b += kPeakBytes;                                                   // a6 peak
  return b;
}

// ------------------------------------------------------------------ contraction
SrcPlan src_plan(const psf_src* h_src, const PatchPlan& plan, const BinRec* rec, const float2* c, float* partial,
                 float* P, const double* dir, const double* peak) {
  SrcPlan p;
  p.peak = peak;
  p.tp = plan.tp;
  p.item0 = 0;
  p.sym = plan.sym ? 1 : 0;
  p.rec = rec;
  p.c = c;
  p.partial = partial;
  p.P = P;
  p.dir = dir;
  p.l0 = h_src->l0;
  p.m0 = h_src->m0;
  p.l_first = h_src->l_first;
  p.m_first = h_src->m_first;
  p.dl = h_src->dl;
  p.dm = h_src->dm;
  p.nl = h_src->nl;
  p.nm = h_src->nm;
  return p;
}

int launch_prec(int prec, int64_t K, bool sym) {
  int kp = prec_base(prec);
  // a few bins: split-BF16's per-term error (3 2^-16 of a term) is not
  // averaged away, so FP32 products run instead (same plan, negligible cost)
  if (kp == PSF_SPLIT_BF16 && K < kSmallK) kp = PSF_FP32;
  // the mixed and stochastic forms need many bins, and exist for the
  // symmetric form only
  if ((kp == PSF_MIXED_FP16 || kp == PSF_SR_FP16) && (K < kMixedMinK || !sym)) kp = PSF_SPLIT_FP16;
  return kp;
}

// (every source of a launch shares the form)
int contraction_prec(int prec, const BatchArgs& a) { return launch_prec(prec, a.K, a.src[0].sym != 0); }

int run_batch(int prec, const BatchArgs& a, int64_t n_wg, hipStream_t s) {
  hipEvent_t ev0;
  hipError_t e;
  if ((e = timed_launch_begin(s, &ev0)) != hipSuccess) return hip_fail(e, "timing event");
  const int kp = contraction_prec(prec, a);
  e = launch_patch(kp, a, n_wg, s);
  if (e != hipSuccess) return hip_fail(e, "k_patch launch");
  if ((e = timed_launch_end(s, ev0)) != hipSuccess) return hip_fail(e, "timing event");
  e = launch_finalize(a, s);
  return e == hipSuccess ? PSF_OK : hip_fail(e, "k_finalize launch");
}

int contract(const psf_obs* obs, const psf_src* h_src, const PatchPlan& plan, int prec, const BinRec* rec,
             const float2* c, float* partial, float* P, hipStream_t s, const double* dir, const double* peak) {
  BatchArgs a;
  a.n_src = 1;
  a.flush_chunks = kFlushChunks;
  a.K = obs->K;
  a.src[0] = src_plan(h_src, plan, rec, c, partial, P, dir, peak);
  a.n_items = tile_plan_items(plan.tp);
  return run_batch(prec, a, a.n_items, s);
}

// ------------------------------------------------------------------ timing
namespace {
struct Timing {
  std::mutex mu;
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  double ms = 0.0;
  int64_t n = 0;
} g_timing;
}  // namespace

bool timing_on() { return g_timing.on; }

hipError_t timed_launch_begin(hipStream_t s, hipEvent_t* ev0) {
  *ev0 = nullptr;
  if (!g_timing.on) return hipSuccess;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return hipSuccess;
  hipError_t e = hipEventCreate(ev0);
  if (e != hipSuccess) return e;
  return hipEventRecord(*ev0, s);
}

hipError_t timed_launch_end(hipStream_t s, hipEvent_t ev0) {
  if (ev0 == nullptr) return hipSuccess;
  hipEvent_t ev1;
  hipError_t e = hipEventCreate(&ev1);
  if (e != hipSuccess) return e;
  e = hipEventRecord(ev1, s);
  std::lock_guard<std::mutex> lock(g_timing.mu);
  g_timing.pending.emplace_back(ev0, ev1);
  return e;
}

}  // namespace psf

using namespace psf;

// ====================================================================== ABI
extern "C" {

const char* psf_version(void) { return "psfdecorr 0.1 gfx950"; }

const char* psf_strerror(int status) {
  switch (status) {
    case PSF_OK: return "ok";
    case PSF_EINVAL: return "invalid argument";
    case PSF_EWORKSPACE: return "workspace missing or too small";
    case PSF_EDEVICE: return "HIP device or launch error";
    case PSF_EUNSUPPORTED: return "unsupported device or feature";
    default: return "unknown status";
  }
}

const char* psf_last_error(void) { return g_msg; }

int psf_timing_enable(int on) {
  std::lock_guard<std::mutex> lock(g_timing.mu);
  g_timing.on = on != 0;
  return PSF_OK;
}

int psf_timing_read(double* ms_total, int64_t* launches) {
  if (!ms_total || !launches) return fail(PSF_EINVAL, "NULL output");
  std::lock_guard<std::mutex> lock(g_timing.mu);
  for (auto& pr : g_timing.pending) {
    hipError_t e = hipEventSynchronize(pr.second);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    g_timing.ms += ms;
    g_timing.n += 1;
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  g_timing.pending.clear();
  *ms_total = g_timing.ms;
  *launches = g_timing.n;
  g_timing.ms = 0.0;
  g_timing.n = 0;
  return PSF_OK;
}

int psf_workspace_bytes(const psf_obs* obs, int32_t n_src, const psf_src* h_srcs, int prec, size_t* out) {
  clear_error();
  int st;
  if ((st = validate_obs(obs)) != PSF_OK) return st;
  if ((st = validate_prec(prec)) != PSF_OK) return st;
  prec = prec_base(prec);  // the normalisation's peak is part of every layout
  if (out == nullptr) return fail(PSF_EINVAL, "out is NULL");
  if (n_src < 1 || h_srcs == nullptr) return fail(PSF_EINVAL, "need n_src >= 1 sources");
  size_t need = 0;
  for (int s = 0; s < n_src; ++s) {
    if ((st = validate_src(&h_srcs[s], s)) != PSF_OK) return st;
    const PatchPlan p = plan_patch(obs, &h_srcs[s], prec, kTargetWorkgroups);
    need = std::max(need, patch_workspace(obs, p));
  }
  need = std::max(need, batched_workspace(obs, n_src, h_srcs, prec));
  need = std::max(need, backward_workspace(obs, n_src, h_srcs, prec));
  need = std::max(need, fullw_workspace(obs, n_src, h_srcs, prec));
  *out = need;
  return PSF_OK;
}

int psf_decorr(const psf_obs* obs, double l0, double m0, float* D, void* stream) {
  clear_error();
  int st;
  if ((st = validate_obs(obs)) != PSF_OK) return st;
  if (!std::isfinite(l0) || !std::isfinite(m0) || l0 * l0 + m0 * m0 >= 1.0)
    return fail(PSF_EINVAL, "bad direction (%g, %g)", l0, m0);
  if (D == nullptr && obs->K > 0) return fail(PSF_EINVAL, "D is NULL");
  if ((st = check_device()) != PSF_OK) return st;
  if (obs->K == 0) return PSF_OK;
  hipError_t e = launch_decorr(view(obs), l0, m0, 0.0, 0.0, nullptr, reinterpret_cast<float2*>(D), nullptr,
                               nullptr, nullptr, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? PSF_OK : hip_fail(e, "k_decorr launch");
}

int psf_decorr_sinc(const psf_obs* obs, double l0, double m0, float* D, void* stream) {
  clear_error();
  int st;
  if ((st = validate_obs(obs)) != PSF_OK) return st;
  if (!std::isfinite(l0) || !std::isfinite(m0) || l0 * l0 + m0 * m0 >= 1.0)
    return fail(PSF_EINVAL, "bad direction (%g, %g)", l0, m0);
  if (D == nullptr && obs->K > 0) return fail(PSF_EINVAL, "D is NULL");
  if (obs->win_t != nullptr || obs->win_c != nullptr)
    return fail(PSF_EINVAL, "Method 1 is the closed form of boxcar averaging: the observation has windows");
  if ((st = check_device()) != PSF_OK) return st;
  if (obs->K == 0) return PSF_OK;
  hipError_t e = launch_decorr_sinc(view(obs), l0, m0, reinterpret_cast<float2*>(D), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? PSF_OK : hip_fail(e, "k_decorr_sinc launch");
}

int psf_patch(const psf_obs* obs, const psf_src* h_src, const float* D, int prec, float* P, void* ws,
              size_t ws_bytes, void* stream) {
  clear_error();
  int st;
  if ((st = validate_obs(obs)) != PSF_OK) return st;
  if ((st = validate_src(h_src, 0)) != PSF_OK) return st;
  if ((st = validate_prec(prec)) != PSF_OK) return st;
  const bool norm = prec_normalise(prec);
  prec = prec_base(prec);
  if (P == nullptr) return fail(PSF_EINVAL, "P is NULL");
  const PatchPlan plan = plan_patch(obs, h_src, prec, kTargetWorkgroups);
  const size_t need = patch_workspace(obs, plan);
  if (ws == nullptr || ws_bytes < need)
    return fail(PSF_EWORKSPACE, "psf_patch needs %zu workspace bytes, got %zu", need, ws_bytes);
  if ((st = check_device()) != PSF_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);

  uint8_t* w = static_cast<uint8_t*>(ws);
  BinRec* rec = reinterpret_cast<BinRec*>(w);
  w += align_up(static_cast<size_t>(obs->K) * sizeof(BinRec), 256);
  float2* c = reinterpret_cast<float2*>(w);
  w += align_up(static_cast<size_t>(obs->K) * sizeof(float2), 256);
  float* partial = reinterpret_cast<float*>(w);
  w += align_up(plan.partial_elems * sizeof(float), 256);
  double* peak = reinterpret_cast<double*>(w);  // [0]: the peak; [1..]: its reduction scratch

  hipError_t e = hipSuccess;
  if (obs->K > 0) {
    e = launch_decorr(view(obs), h_src->l0, h_src->m0, h_src->dl, h_src->dm, reinterpret_cast<const float2*>(D),
                      nullptr, rec, c, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "k_decorr launch");
  }
  if (norm && (e = launch_peak(c, obs->K, peak + 1, peak, s)) != hipSuccess) return hip_fail(e, "peak launch");
  return contract(obs, h_src, plan, prec, rec, c, partial, P, s, nullptr, norm ? peak : nullptr);
}

}  // extern "C"
// ====================================================================== no-allocation variant
namespace psf {
namespace {
// Scratch of psf_patch_noalloc: one array per GPU, in the library's code
// object, held until the process ends.  320 MiB holds the per-bin records
// (40 bytes per bin), partial slabs and peak of one patch: K up to about
// 6.5 million bins at 257 x 257, more for smaller patches.
constexpr size_t kNoAllocScratchBytes = size_t(320) << 20;
__device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

// Device address of this device's copy of `scratch`, resolved once per
// device with that device current.  In host code the array's name is only
// a host-side stand-in: every kernel argument uses the resolved address.
int scratch_address(void** out) {
  static std::mutex mu;
  static std::vector<void*> addr;  // per device
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(mu);
  if (static_cast<int>(addr.size()) <= dev) addr.resize(dev + 1, nullptr);
  if (addr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    addr[dev] = p;
  }
  *out = addr[dev];
  return PSF_OK;
}
}  // namespace
}  // namespace psf

extern "C" int psf_patch_noalloc(const psf_obs* obs, const psf_src* h_src, const float* D, int prec, float* P,
                                 void* stream) {
  clear_error();
  int st;
  if ((st = validate_obs(obs)) != PSF_OK) return st;
  if ((st = validate_src(h_src, 0)) != PSF_OK) return st;
  if ((st = validate_prec(prec)) != PSF_OK) return st;
  if (P == nullptr) return fail(PSF_EINVAL, "P is NULL");
  const size_t need = patch_workspace(obs, plan_patch(obs, h_src, prec_base(prec), kTargetWorkgroups));
  if (need > kNoAllocScratchBytes)
    return fail(PSF_EWORKSPACE,
                "psf_patch_noalloc needs %zu bytes of scratch for this observation and patch; its fixed scratch "
                "holds %zu (use psf_patch with a workspace)",
                need, kNoAllocScratchBytes);
  if ((st = check_device()) != PSF_OK) return st;
  void* ws = nullptr;
  if ((st = scratch_address(&ws)) != PSF_OK) return st;
  // psf_patch on the library's scratch: nothing in it needs to start at zero
  // (every partial slab, record and peak is written before it is read)
  return psf_patch(obs, h_src, D, prec, P, ws, kNoAllocScratchBytes, stream);
}
