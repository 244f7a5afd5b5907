// Kernel-facing argument blocks and launchers of libpsfdecorr.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psf {

// Device view of an observation (all pointers device memory).
struct ObsView {
  const double* uvw;      // [n_bl][n_t][3]
  const double* freq;     // [n_ch]
  const int32_t* bl_bin;  // [n_bl][2]
  const int64_t* koff;    // [n_bl + 1]
  const int64_t* tboff;   // [n_bl + 1]
  const double* uvw_c;    // [n_tb][3]
  const float* W;         // [K]
  int64_t K;
  int64_t n_tb;
  int n_bl, n_t, n_ch;
};

enum Prec : int { kFP32 = 0, kSplitBF16 = 1, kSplitFP16 = 2, kPlainBF16 = 3 };

// One source's patch contraction over precomputed per-bin records.
struct PatchArgs {
  const double2* uvp;    // [K] (u'_k, v'_k) in wavelengths
  const float2* c;       // [K] W_k D_k
  int64_t K;
  double l_first, dl, l0;
  double m_first, dm, m0;
  int nl, nm;            // patch size
  int nbi, nbj;          // 16-pixel blocks along l and m
  int tiles_i, tiles_j;  // tiles of the patch, each handled by one workgroup per k-slice
  int n_split;           // k-slices
  int64_t k_per_split;   // multiple of the chunk length
  float* partial;        // [n_split][16 nbi][16 nbj]
};

// Geometry of a contraction kernel instance (compile-time constants exposed
// to the host planner).
struct PatchShape {
  int waves_m, waves_n;    // wave grid of a workgroup
  int blk_m, blk_n;        // max 16x16 blocks per wave
  int kchunk;              // visibilities per LDS chunk
};

hipError_t launch_decorr(const ObsView& o, double l0, double m0, const float2* D_in, float2* D_out,
                         double2* uvp_out, float2* c_out, float2* dDl_out, float2* dDm_out,
                         hipStream_t stream);

PatchShape patch_shape(int prec);
hipError_t launch_patch(int prec, const PatchArgs& a, hipStream_t stream);
hipError_t launch_finalize(const float* partial, int n_split, int nbi, int nbj, int nl, int nm,
                           float* P, hipStream_t stream);

}  // namespace psf
