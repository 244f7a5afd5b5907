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
  const float* win_t;     // [n_bl][n_t] or null (boxcar in time)
  const float* win_c;     // [n_bl][n_ch] or null (boxcar in frequency)
  int64_t K;
  int64_t n_tb;
  int n_bl, n_t, n_ch;
};

// Per-bin record of one source that the contraction streams: the w-shifted
// bin-centre coordinates and the phase factors of a 16-pixel step along each
// axis of the source's pixel grid, exp(2 pi i u' 16 dl) and
// exp(2 pi i v' 16 dm).
struct BinRec {
  double up, vp;          // u'_k, v'_k in wavelengths
  float2 step_a, step_b;  // FP64-reduced, FP32 sin/cos
};

// kMixedFP16: symmetric form only; the row operand (cos and sin) is one FP16
// value, rounded stochastically, the column operand is split hi + lo in
// FP16 (two products).  kSRFP16: symmetric form only; both operands one
// stochastically rounded FP16 value each (one product).
enum Prec : int { kFP32 = 0, kSplitBF16 = 1, kSplitFP16 = 2, kPlainBF16 = 3, kMixedFP16 = 4, kSRFP16 = 5 };

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

// Per-source part of a contraction launch.  A launch contracts the patches
// of up to kMaxBatch sources of one tile family; its work items (tile,
// k-slice) are numbered source by source (src[s].item0 is the first item of
// source s) and tile by tile within a source as TilePlan describes.
struct SrcPlan {
  TilePlan tp;
  int64_t item0;
  // 1: the patch is 65, 129 or 257 rows high and the contraction runs in
  // its symmetric form (rows of cos and sin of the non-negative half of the
  // row offsets from the grid's centre row, inner dimension K; see
  // k_patch.hip).  Every source of a launch agrees.
  int sym;
  const BinRec* rec;  // [K] per-bin records
  const float2* c;     // [K] W_k D_k (or an adjoint coefficient vector)
  float* partial;      // partial slabs, see TilePlan
  float* P;            // output patch [nl][nm]
  // If not null: the patch's value at the source, 2 Re sum_k c_k (FP64,
  // written by launch_peak before the finalise), which divides the output.
  const double* peak;
  // Source direction and pixel grid: read at run time from `dir` (device
  // memory laid out as psf_src: l0, m0, l_first, m_first, dl, dm) when it
  // is not null, else taken from the fields below.
  const double* dir;
  double l0, m0, l_first, m_first, dl, dm;
  int nl, nm;
};

constexpr int kMaxBatch = 16;

struct BatchArgs {
  int n_src;
  int flush_chunks;  // chunks per first-level (matrix-core) accumulation run
  int64_t K;
  int64_t n_items;
  SrcPlan src[kMaxBatch];
};

constexpr int kPatchChunk = 16;     // visibilities per contraction chunk
constexpr int kPatchChunkSym = 32;  // visibilities per chunk of the symmetric form

// Power-of-two scale of the adjoint coefficient vectors (keeps them inside
// the FP16 range; exact in every precision).
constexpr double kAdjointScale = 1.0 / 4096.0;

// coef_out (optional, [5][K]): the adjoint coefficient vectors e0..e4 (see
// k_decorr.hip) times kAdjointScale; needs D_in == nullptr.
// dir (optional): device memory laid out as psf_src (l0, m0, l_first,
// m_first, dl, dm) from which the direction and cells are read at run time
// instead of l0, m0, dl, dm.
hipError_t launch_decorr(const ObsView& o, double l0, double m0, double dl, double dm, const float2* D_in,
                         float2* D_out, BinRec* rec_out, float2* c_out, float2* coef_out, hipStream_t stream,
                         const double* dir = nullptr);
// Method-1 (sinc) decorrelation factors, written as (D, 0).
hipError_t launch_decorr_sinc(const ObsView& o, double l0, double m0, float2* D_out, hipStream_t stream);
// Records of n_src sources in one launch: source y's direction and grid are
// read from device memory (dirs + y dir_stride, laid out as psf_src: l0, m0,
// l_first, m_first, dl, dm), its records are written at
// rec_out / c_out + y rec_stride.
hipError_t launch_decorr_sources(const ObsView& o, const double* dirs, int64_t dir_stride, int n_src,
                                 BinRec* rec_out, float2* c_out, int64_t rec_stride, hipStream_t stream);
// dLoss/d(l0, m0) of one source from G = dLoss/dP and the five derivative
// patches Pe [5][nl][nm] of the coefficient vectors e0..e4, FP64, written
// to grad[0..1].
hipError_t launch_grad_reduce(const float* G, const float* Pe, int nl, int nm, double l_first, double dl,
                              double l0, double m_first, double dm, double m0, double* grad, hipStream_t stream,
                              const double* dir = nullptr);

// Tile shapes of the compiled contraction for a patch of nbi x nbj blocks;
// fills tbi, tbj and the tile counts of *tp (not ns / kps).
void plan_tiles(int nbi, int nbj, TilePlan* tp);
// Whether a patch of nl x nm pixels has a compiled symmetric form (nl is
// 65, 129 or 257 and nm falls in the same tile family).
bool sym_patch_size(int nl, int nm);
// Contraction workgroups one compute unit runs at once for this tile plan
// and launch precision (its kernel's occupancy): 2 for the 5 x 5 block tiles
// and for the stochastic form, else 1.
int tile_wgs_per_cu(const TilePlan& t, int prec);
// Blocks of the busiest SIMD (its two contraction waves) of a tbi x tbj tile.
int tile_max_simd_blocks(int tbi, int tbj, bool sym);
size_t tile_plan_partial_elems(const TilePlan& tp);
// Work items of one source's tile plan.
int64_t tile_plan_items(const TilePlan& tp);
// Contraction of every item of `a` with `grid` persistent workgroups (each
// takes items blockIdx.x, blockIdx.x + grid, ...).
hipError_t launch_patch(int prec, const BatchArgs& a, int64_t grid, hipStream_t stream);
// P = 2 * (sum of the k-slices) for every source of `a` (divided by the
// source's peak where SrcPlan::peak is set).
hipError_t launch_finalize(const BatchArgs& a, hipStream_t stream);

// Normalisation [section 4: errors are taken on PSFs normalised at the
// source]: peak = 2 Re sum_k c_k of one source, FP64, summed in a fixed
// order (kPeakBlocks contiguous ranges, then their partial sums in order).
// scratch holds kPeakBlocks doubles.
constexpr int kPeakBlocks = 512;
hipError_t launch_peak(const float2* c, int64_t K, double* scratch, double* peak, hipStream_t stream);

}  // namespace psf
