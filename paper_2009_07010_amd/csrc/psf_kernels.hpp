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

// Tiling of one patch.  Row tiles come in two heights (ti_a tiles of tbi[0]
// blocks, then ti_b tiles of tbi[1]), column tiles in two widths (tj_a of
// tbj[0], then tj_b of tbj[1]); a 16x16 block is the unit.  Each tile type
// (row type r, column type c) gets ns[r][c] k-slices of kps[r][c]
// visibilities.  Workgroups, and the partial slabs they write
// ([16 tbi][16 tbj] floats each), are numbered tile by tile in row-major
// tile order, slice by slice within a tile.
struct TilePlan {
  int tbi[2], tbj[2];
  int ti_a, ti_b, tj_a, tj_b;
  int ns[2][2];
  int64_t kps[2][2];
};

// One source's patch contraction over precomputed per-bin records.
struct PatchArgs {
  const double2* uvp;        // [K] (u'_k, v'_k) in wavelengths
  const float2* c;           // [K] W_k D_k
  int64_t K;
  double l_first, dl, l0;
  double m_first, dm, m0;
  int nl, nm;                // patch size
  TilePlan tp;
  int flush_chunks;          // chunks per first-level (matrix-core) accumulation run
  float* partial;            // partial slabs, see TilePlan
};

constexpr int kPatchChunk = 16;  // visibilities per contraction chunk

// Power-of-two scale of the adjoint coefficient vectors (keeps them inside
// the FP16 range; exact in every precision).
constexpr double kAdjointScale = 1.0 / 4096.0;

// coef_out (optional, [5][K]): the adjoint coefficient vectors e0..e4 (see
// k_decorr.hip) times kAdjointScale; needs D_in == nullptr.
hipError_t launch_decorr(const ObsView& o, double l0, double m0, const float2* D_in, float2* D_out,
                         double2* uvp_out, float2* c_out, float2* coef_out, hipStream_t stream);
// dLoss/d(l0, m0) of one source from G = dLoss/dP and the five derivative
// patches Pe [5][nl][nm] of the coefficient vectors e0..e4, FP64, written
// to grad[0..1].
hipError_t launch_grad_reduce(const float* G, const float* Pe, int nl, int nm, double l_first, double dl,
                              double l0, double m_first, double dm, double m0, double* grad, hipStream_t stream);

// Tile shapes of the compiled contraction for a patch of nbi x nbj blocks;
// fills tbi, tbj and the tile counts of *tp (not ns / kps).
void plan_tiles(int nbi, int nbj, TilePlan* tp);
int64_t tile_plan_workgroups(const TilePlan& tp);
// Blocks of the busiest SIMD (its two contraction waves) of a tbi x tbj tile.
int tile_max_simd_blocks(int tbi, int tbj);
size_t tile_plan_partial_elems(const TilePlan& tp);
hipError_t launch_patch(int prec, const PatchArgs& a, hipStream_t stream);
hipError_t launch_finalize(const PatchArgs& a, float* P, hipStream_t stream);

}  // namespace psf
