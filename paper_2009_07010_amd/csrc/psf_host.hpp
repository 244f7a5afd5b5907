// Host-side helpers shared by the ABI translation units of libpsfdecorr.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/psf.h"
#include "psf_kernels.hpp"

namespace psf {

// Workgroups one contraction launch aims for: one per compute unit of an
// MI355X (256 CUs), the contraction kernels running one workgroup per CU.
constexpr int kTargetWorkgroups = 256;
// First-level accumulation run of the contraction: 128 chunks of 16
// visibilities (2048 terms per pixel) before folding into the second level.
constexpr int kFlushChunks = 128;
// Below this many bins the split-BF16 contraction runs as FP32.
constexpr int64_t kSmallK = 256;
// Below this many bins (and for patches without a symmetric form) the mixed
// and stochastic FP16 contractions run as split-FP16: their single-FP16
// roundings average out only over many visibilities.
constexpr int64_t kMixedMinK = int64_t(1) << 18;

struct PatchPlan {
  TilePlan tp;
  size_t partial_elems;
  bool sym;  // symmetric form of the contraction (see k_patch.hip)
};

// Whether a source's contraction runs in the symmetric form: a patch size
// with a compiled symmetric form (any grid position: the offset of the
// grid's centre row from the source joins the coefficients).
bool sym_source(const psf_src* s);

int fail(int status, const char* fmt, ...);
// Clears the thread's last-error message (every entry point starts with it).
void clear_error();
int hip_fail(hipError_t e, const char* what);
int check_device();
int validate_obs(const psf_obs* o);
int validate_src(const psf_src* s, int idx);
// Accepts the arithmetic with or without PSF_NORMALISE (entry points that
// cannot normalise check the flag themselves); prec_base strips the flag.
int validate_prec(int prec);
inline int prec_base(int prec) { return prec & ~PSF_NORMALISE; }
inline bool prec_normalise(int prec) { return (prec & PSF_NORMALISE) != 0; }
int reject_normalise(int prec, const char* entry);
// Workspace bytes of one source's peak (a6) and its reduction scratch.
constexpr size_t kPeakBytes = 256 * ((8 * (kPeakBlocks + 1) + 255) / 256);
ObsView view(const psf_obs* o);
size_t align_up(size_t x, size_t a);
// Matrix-core / generator cost of a source's whole patch (SIMD cycles).
double patch_work(const psf_obs* o, const psf_src* s, int prec);
// Tile plan whose work items each cost about item_work.
PatchPlan plan_patch_items(const psf_obs* o, const psf_src* s, int prec, double item_work);
// Tile plan with about target_wgs work items.
PatchPlan plan_patch(const psf_obs* o, const psf_src* s, int prec, int target_wgs);
size_t patch_workspace(const psf_obs* o, const PatchPlan& p);
// The precision a contraction runs in for the caller's prec, K bins and
// form (small K and non-symmetric patches change it, see kSmallK,
// kMixedMinK); contraction_prec for the sources of a launch.
int launch_prec(int prec, int64_t K, bool sym);
int contraction_prec(int prec, const BatchArgs& a);

// The contraction and finalise of one patch from per-bin records (u', v')
// and coefficients c (c_k = W_k D_k for the patch itself).
// dir (optional): the source's direction and grid in device memory
// (psf_src layout), read at run time instead of h_src's.
// One Method-2 patch (psf_method2_patch's arithmetic) with its direction
// read from device memory at d_dir (l0, m0); work: N^2 complex values.
int method2_patch_device_dir(int32_t N, double cell, const float* S, const double* d_dir, double dt_bin,
                             double dnu_bin, double nu, float* P, float2* work, hipStream_t s);

int contract(const psf_obs* obs, const psf_src* h_src, const PatchPlan& plan, int prec, const BinRec* rec,
             const float2* c, float* partial, float* P, hipStream_t s, const double* dir = nullptr,
             const double* peak = nullptr);

SrcPlan src_plan(const psf_src* h_src, const PatchPlan& plan, const BinRec* rec, const float2* c, float* partial,
                 float* P, const double* dir, const double* peak = nullptr);
// Contraction (n_wg persistent workgroups) and finalise of the sources of a.
int run_batch(int prec, const BatchArgs& a, int64_t n_wg, hipStream_t s);

size_t batched_workspace(const psf_obs* o, int n_src, const psf_src* h_srcs, int prec);
size_t backward_workspace(const psf_obs* o, int n_src, const psf_src* h_srcs, int prec);
size_t fullw_workspace(const psf_obs* o, int n_src, const psf_src* h_srcs, int prec);
// Reverse-mode adjoint (k_adjoint.hip): whether it serves this source and
// precision, the bytes of its per-workgroup partial sums, and the launch
// (workgroup partials, then their fixed-order sum into grad[0..1]).
bool adjoint_reverse_ok(int prec, const psf_obs* o, const psf_src& s);
size_t adjoint_reverse_partial_bytes();
hipError_t launch_adjoint_reverse(const psf_obs* o, const psf_src& s, int prec, const BinRec* rec,
                                  const float2* coef, const float* G, double* partial, double* grad,
                                  hipStream_t st, const double* dir = nullptr);

bool timing_on();
hipError_t timed_launch_begin(hipStream_t s, hipEvent_t* ev0);
hipError_t timed_launch_end(hipStream_t s, hipEvent_t ev0);

}  // namespace psf
