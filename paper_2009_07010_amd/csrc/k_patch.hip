// K-b + K-c/K-e + K-f: phase-factor generation, matrix-core patch
// contraction and the fixed-order split-K finalise.
//
// The patch P_ij = 2 Re sum_k c_k a_ki b_kj, with c_k = W_k D_k,
// a_ki = exp(2 pi i u'_k x_i) and b_kj = exp(2 pi i v'_k y_j), is a real
// matrix product over an inner dimension of 2K:
//   A[k'][i] = (Re(c a), -Im(c a)) = conj(c_k a_ki),  B[k'][j] = (Re b, Im b)
//   P = 2 A^T B.
// The inner dimension runs over visibilities (millions), the output is a
// small patch, so each workgroup owns one output tile and one contiguous
// k-slice, keeps the tile in matrix-core accumulators, and writes a partial
// tile; K-f adds the partials in slice order (deterministic).
//
// Per chunk of 16 visibilities a workgroup of 4 waves
//   * generates the chunk's A and B columns for its tile into one of two LDS
//     buffers, in the exact operand layout of the MFMA instruction (K-b), and
//   * contracts the other buffer's chunk with matrix-core instructions (K-c),
// so one barrier per chunk separates writers from readers.  Each thread of
// the generator owns one visibility and one run of R consecutive rows: one
// FP64-reduced seed exp(2 pi i u' x_run) and one FP64-reduced step
// exp(2 pi i u' dl), then FP32 complex multiplication along the run.
//
// Tile and wave shapes are compile-time: a tile of TBI x TBJ 16x16 blocks is
// cut into a 2 x 2 grid of wave sub-tiles whose block counts differ by at
// most one; each wave runs the loop instantiated for its own shape (chosen
// by a uniform switch on the wave index), so the contraction is straight-line
// code with no per-block conditions.
//
// Two-level accumulation: matrix-core accumulators collect a run of
// flush_chunks chunks and are then added into a second FP32 tile held in
// registers.  A single FP32 accumulator over a whole k-slice loses up to
// ~2e-5 of the peak at pixels where many nearly equal terms add up (the
// rounding of a long sum of similar increments is coherent); short runs
// keep each rounding small relative to the final value.
//
// Split forms: every operand value v is stored as hi = round16(v) and
// lo = round16(v - hi); the product uses hi*hi + hi*lo + lo*hi (three MFMAs)
// with FP32 accumulation.
#include "psf_device.hpp"
#include "psf_kernels.hpp"

namespace psf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// LDS byte pointer (address space 3), so that every operand access is a
// ds_read / ds_write with a 32-bit address rather than a flat access.
typedef __attribute__((address_space(3))) uint8_t lds_t;

// One LDS operand row: 32 16-bit values (16 visibilities x re/im) or, per
// group of 8 visibilities, 16 floats: 64 bytes, padded to 80 so that 8
// consecutive rows read with 16-byte loads touch 32 distinct banks.
constexpr int kRowBytes = 80;
constexpr int kChunk = 16;  // visibilities per LDS chunk

// Generator geometry of a tile of TI x TJ pixels: run length R such that the
// A runs and B runs together number at most 16 (16 runs x 16 visibilities =
// 256 threads).
constexpr int gen_run(int TI, int TJ) {
  int R = (TI + TJ + 15) / 16;
  while ((TI + R - 1) / R + (TJ + R - 1) / R > 16) ++R;
  return R;
}

template <int PREC>
__device__ __forceinline__ f32x4 mfma16(const bf16x8& a, const bf16x8& b, f32x4 acc) {
  if constexpr (PREC == kSplitFP16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b),
                                                  acc, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
}

// Store one complex operand value of visibility v (0..15) at `row` of a
// plane.  FP32: two groups of 8 visibilities, group stride gstride; lane
// group g of the 16x16x4 instruction takes k' = g of each of its four
// k-steps, i.e. (re v0, im v0, re v1, im v1) of the step's two visibilities.
// 16-bit: lane group g of the 16x16x32 instruction takes k' = 8g..8g+7,
// i.e. visibilities 4g..4g+3 as (re, im) pairs.
template <int PREC>
__device__ __forceinline__ void store_operand(lds_t* hi_plane, int lo_off, int gstride, int row, int v, cf32 z) {
  if constexpr (PREC == kFP32) {
    const int g = v >> 3, kv = v & 7;
    lds_t* p = hi_plane + g * gstride + row * kRowBytes + (kv & 1) * 32 + (kv >> 1) * 4;
    *reinterpret_cast<__attribute__((address_space(3))) float*>(p) = z.re;
    *reinterpret_cast<__attribute__((address_space(3))) float*>(p + 16) = z.im;
  } else {
    lds_t* p = hi_plane + row * kRowBytes + v * 4;
    uint32_t hi, lo = 0;
    if constexpr (PREC == kSplitFP16) {
      hi = pack_f16x2(z.re, z.im);
      lo = pack_f16x2(z.re - f16_lo_to_f32(hi), z.im - f16_hi_to_f32(hi));
    } else {
      hi = pack_bf16x2(z.re, z.im);
      if constexpr (PREC == kSplitBF16) lo = pack_bf16x2(z.re - bf16_lo_to_f32(hi), z.im - bf16_hi_to_f32(hi));
    }
    *reinterpret_cast<__attribute__((address_space(3))) uint32_t*>(p) = hi;
    if constexpr (PREC != kPlainBF16) *reinterpret_cast<__attribute__((address_space(3))) uint32_t*>(p + lo_off) = lo;
  }
}

// LDS geometry of one tile type.
template <int PREC, int TBI, int TBJ>
struct TileGeom {
  static constexpr int TI = 16 * TBI, TJ = 16 * TBJ;
  static constexpr int R = gen_run(TI, TJ);
  static constexpr int NA = (TI + R - 1) / R, NB = (TJ + R - 1) / R;
  static constexpr int ROWS_A = NA * R, ROWS_B = NB * R;  // rows written (>= TI, TJ)
  static constexpr bool F32 = PREC == kFP32;
  static constexpr bool TWO = PREC == kSplitBF16 || PREC == kSplitFP16;
  static constexpr int GA = ROWS_A * kRowBytes, GB = ROWS_B * kRowBytes;  // one group / plane
  static constexpr int APL = (F32 ? 2 : 1) * GA, BPL = (F32 ? 2 : 1) * GB;
  static constexpr int NPL = TWO ? 2 : 1;
  static constexpr int BUF = NPL * (APL + BPL);
  static constexpr int LDS = 2 * BUF;
};

// The whole k-loop of one wave whose sub-tile is M x N blocks starting at
// block (WI0, WJ0) of the tile.
template <int PREC, int TBI, int TBJ, int M, int N, int WI0, int WJ0>
__device__ __forceinline__ void wave_loop(const PatchArgs& a, lds_t* smem, int bi0, int bj0, int64_t kb,
                                          int64_t ke, float* __restrict__ out, int width) {
  using G = TileGeom<PREC, TBI, TBJ>;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t nch = ke > kb ? (ke - kb + kChunk - 1) / kChunk : 0;

  // generator role: visibility gv of each chunk, run grho of A rows then B rows
  const int gv = tid & 15, grho = tid >> 4;
  const bool gA = grho < G::NA;
  const bool gact = grho < G::NA + G::NB;
  const int grow0 = (gA ? grho : grho - G::NA) * G::R;
  const double gpos0 = gA ? (a.l_first + (16 * bi0 + grow0) * a.dl) - a.l0
                          : (a.m_first + (16 * bj0 + grow0) * a.dm) - a.m0;
  const double gd = gA ? a.dl : a.dm;
  const int gstride = gA ? G::GA : G::GB;
  const int goff = gA ? 0 : G::NPL * G::APL;
  const int glo = gA ? G::APL : G::BPL;

  auto fetch = [&](int64_t n, double& f, cf32& cc) {
    f = 0.0;
    cc = {0.f, 0.f};
    const int64_t kg = kb + n * kChunk + gv;
    if (gact && kg < ke) {
      const double2 uv = a.uvp[kg];
      f = gA ? uv.x : uv.y;
      const float2 c = a.c[kg];
      cc = {c.x, c.y};
    }
  };
  auto generate = [&](int buf, double f, cf32 cc) {
    if (!gact) return;
    cf32 z = expi_turns(f * gpos0);
    cf32 zs = expi_turns(f * gd);
    if (gA) {
      z = conj(cmul(cc, z));
      zs = conj(zs);
    }
    lds_t* plane = smem + buf * G::BUF + goff;
#pragma unroll
    for (int q = 0; q < G::R; ++q) {
      store_operand<PREC>(plane, glo, gstride, grow0 + q, gv, z);
      z = cmul(z, zs);
    }
  };

  f32x4 acc[M][N], tot[M][N];
#pragma unroll
  for (int r = 0; r < M; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) {
      acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
      tot[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

  if (nch > 0) {
    double f;
    cf32 cc;
    fetch(0, f, cc);
    generate(0, f, cc);
  }
  __syncthreads();

  // Runs of flush_chunks chunks: matrix-core accumulators within a run, the
  // second-level tile between runs.  The last chunk also generates a chunk
  // past the end (all-zero weights) into the idle buffer; nothing reads it.
  const int64_t flush = a.flush_chunks;
  for (int64_t run0 = 0; run0 < nch; run0 += flush) {
    const int64_t run1 = min(nch, run0 + flush);
    for (int64_t n = run0; n < run1; ++n) {
      const int cur = static_cast<int>(n & 1);
      double fn;
      cf32 ccn;
      fetch(n + 1, fn, ccn);

      // ---- K-c / K-e: contract the current chunk
      const lds_t* Ah = smem + cur * G::BUF;
      const lds_t* Bh = Ah + G::NPL * G::APL;
      if constexpr (G::F32) {
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          f32x4 av[M];
#pragma unroll
          for (int r = 0; r < M; ++r)
            av[r] = *reinterpret_cast<const __attribute__((address_space(3))) f32x4*>(
                Ah + g * G::GA + (16 * (WI0 + r) + lr) * kRowBytes + lg * 16);
#pragma unroll
          for (int c = 0; c < N; ++c) {
            const f32x4 bv = *reinterpret_cast<const __attribute__((address_space(3))) f32x4*>(
                Bh + g * G::GB + (16 * (WJ0 + c) + lr) * kRowBytes + lg * 16);
#pragma unroll
            for (int r = 0; r < M; ++r)
#pragma unroll
              for (int e = 0; e < 4; ++e)
                acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r][e], bv[e], acc[r][c], 0, 0, 0);
          }
        }
      } else {
        bf16x8 ah[M], al[M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
          const int off = (16 * (WI0 + r) + lr) * kRowBytes + lg * 16;
          ah[r] = *reinterpret_cast<const __attribute__((address_space(3))) bf16x8*>(Ah + off);
          if constexpr (G::TWO)
            al[r] = *reinterpret_cast<const __attribute__((address_space(3))) bf16x8*>(Ah + G::APL + off);
        }
#pragma unroll
        for (int c = 0; c < N; ++c) {
          const int off = (16 * (WJ0 + c) + lr) * kRowBytes + lg * 16;
          const bf16x8 bh = *reinterpret_cast<const __attribute__((address_space(3))) bf16x8*>(Bh + off);
          bf16x8 bl;
          if constexpr (G::TWO) bl = *reinterpret_cast<const __attribute__((address_space(3))) bf16x8*>(Bh + G::BPL + off);
#pragma unroll
          for (int r = 0; r < M; ++r) {
            acc[r][c] = mfma16<PREC>(ah[r], bh, acc[r][c]);
            if constexpr (G::TWO) {
              acc[r][c] = mfma16<PREC>(ah[r], bl, acc[r][c]);
              acc[r][c] = mfma16<PREC>(al[r], bh, acc[r][c]);
            }
          }
        }
      }

      // ---- K-b: phase factors of the next chunk into the other buffer
      generate(cur ^ 1, fn, ccn);
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
      for (int c = 0; c < N; ++c) {
        tot[r][c] += acc[r][c];
        acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
  }

  // ---- partial tile of this k-slice (rows/cols beyond the patch are padding)
#pragma unroll
  for (int r = 0; r < M; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const int col = 16 * (WJ0 + c) + lr;  // tile-local
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = 16 * (WI0 + r) + 4 * lg + e;  // tile-local row
        out[static_cast<size_t>(row) * width + col] = tot[r][c][e];
      }
    }
}

template <int PREC, int TBI, int TBJ>
__device__ __forceinline__ void tile_body(const PatchArgs& a, lds_t* smem, int bi0, int bj0, int64_t kb,
                                          int64_t ke, float* out, int width) {
  constexpr int M0 = (TBI + 1) / 2, M1 = TBI / 2, N0 = (TBJ + 1) / 2, N1 = TBJ / 2;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  switch (wave) {
    case 0: wave_loop<PREC, TBI, TBJ, M0, N0, 0, 0>(a, smem, bi0, bj0, kb, ke, out, width); break;
    case 1: wave_loop<PREC, TBI, TBJ, M0, N1, 0, N0>(a, smem, bi0, bj0, kb, ke, out, width); break;
    case 2: wave_loop<PREC, TBI, TBJ, M1, N0, M0, 0>(a, smem, bi0, bj0, kb, ke, out, width); break;
    default: wave_loop<PREC, TBI, TBJ, M1, N1, M0, N0>(a, smem, bi0, bj0, kb, ke, out, width); break;
  }
}

// ---------------------------------------------------------------- tile plan
__host__ __device__ inline int64_t slab_elems(const TilePlan& t, int r, int c) {
  return 256LL * t.tbi[r] * t.tbj[c];
}
__host__ __device__ inline int64_t row_wgs(const TilePlan& t, int r) {
  return static_cast<int64_t>(t.tj_a) * t.ns[r][0] + static_cast<int64_t>(t.tj_b) * t.ns[r][1];
}
__host__ __device__ inline int64_t row_elems(const TilePlan& t, int r) {
  return static_cast<int64_t>(t.tj_a) * t.ns[r][0] * slab_elems(t, r, 0) +
         static_cast<int64_t>(t.tj_b) * t.ns[r][1] * slab_elems(t, r, 1);
}
// Element offset of the first slab of tile (ti, tj).
__host__ __device__ inline int64_t tile_first_elem(const TilePlan& t, int ti, int tj) {
  const int r = ti < t.ti_a ? 0 : 1;
  const int ra = ti < t.ti_a ? ti : t.ti_a, rb = ti - ra;
  const int ca = tj < t.tj_a ? tj : t.tj_a, cb = tj - ca;
  return ra * row_elems(t, 0) + rb * row_elems(t, 1) + ca * t.ns[r][0] * slab_elems(t, r, 0) +
         cb * t.ns[r][1] * slab_elems(t, r, 1);
}

int64_t tile_plan_workgroups(const TilePlan& t) {
  return t.ti_a * row_wgs(t, 0) + t.ti_b * row_wgs(t, 1);
}
size_t tile_plan_partial_elems(const TilePlan& t) {
  return static_cast<size_t>(t.ti_a * row_elems(t, 0) + t.ti_b * row_elems(t, 1));
}

// The contraction kernel.  Template arguments are the two tile heights and
// the two tile widths (in blocks) of its tile family.
template <int PREC, int I0, int I1, int J0, int J1>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(1, 1)))
void k_patch(PatchArgs a) {
  constexpr int L00 = TileGeom<PREC, I0, J0>::LDS, L01 = TileGeom<PREC, I0, J1>::LDS;
  constexpr int L10 = TileGeom<PREC, I1, J0>::LDS, L11 = TileGeom<PREC, I1, J1>::LDS;
  constexpr int LA = L00 > L01 ? L00 : L01, LB = L10 > L11 ? L10 : L11;
  __shared__ __attribute__((aligned(16))) uint8_t smem_raw[LA > LB ? LA : LB];
  lds_t* smem = (lds_t*)smem_raw;
  const TilePlan& t = a.tp;
  // decode (tile row, tile column, k-slice) from the workgroup index
  int64_t w = blockIdx.x;
  int r, ti;
  int64_t wr;
  const int64_t rwa = row_wgs(t, 0);
  if (w < t.ti_a * rwa) {
    r = 0;
    ti = static_cast<int>(w / rwa);
    wr = w - ti * rwa;
  } else {
    r = 1;
    w -= t.ti_a * rwa;
    const int64_t rwb = row_wgs(t, 1);
    ti = t.ti_a + static_cast<int>(w / rwb);
    wr = w - (ti - t.ti_a) * rwb;
  }
  int c, tj, split;
  const int64_t cwa = static_cast<int64_t>(t.tj_a) * t.ns[r][0];
  if (wr < cwa) {
    c = 0;
    tj = static_cast<int>(wr / t.ns[r][0]);
    split = static_cast<int>(wr - static_cast<int64_t>(tj) * t.ns[r][0]);
  } else {
    c = 1;
    wr -= cwa;
    const int q = static_cast<int>(wr / t.ns[r][1]);
    tj = t.tj_a + q;
    split = static_cast<int>(wr - static_cast<int64_t>(q) * t.ns[r][1]);
  }
  const int bi0 = ti < t.ti_a ? ti * t.tbi[0] : t.ti_a * t.tbi[0] + (ti - t.ti_a) * t.tbi[1];
  const int bj0 = tj < t.tj_a ? tj * t.tbj[0] : t.tj_a * t.tbj[0] + (tj - t.tj_a) * t.tbj[1];
  const int64_t kps = t.kps[r][c];
  const int64_t kb = static_cast<int64_t>(split) * kps;
  const int64_t ke = min(a.K, kb + kps);
  float* out = a.partial + tile_first_elem(t, ti, tj) + static_cast<int64_t>(split) * slab_elems(t, r, c);
  switch (r * 2 + c) {
    case 0: tile_body<PREC, I0, J0>(a, smem, bi0, bj0, kb, ke, out, 16 * J0); break;
    case 1: tile_body<PREC, I0, J1>(a, smem, bi0, bj0, kb, ke, out, 16 * J1); break;
    case 2: tile_body<PREC, I1, J0>(a, smem, bi0, bj0, kb, ke, out, 16 * J0); break;
    default: tile_body<PREC, I1, J1>(a, smem, bi0, bj0, kb, ke, out, 16 * J1); break;
  }
}

// K-f: P = 2 * sum over the k-slices of the pixel's tile, in slice order.
__global__ __launch_bounds__(256) void k_finalize(PatchArgs a, float* __restrict__ P) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(a.nl) * a.nm) return;
  const TilePlan& t = a.tp;
  const int i = static_cast<int>(idx / a.nm), j = static_cast<int>(idx - static_cast<int64_t>(i) * a.nm);
  const int span_i = t.ti_a * 16 * t.tbi[0], span_j = t.tj_a * 16 * t.tbj[0];
  const int r = i < span_i ? 0 : 1, c = j < span_j ? 0 : 1;
  const int hi = 16 * t.tbi[r], wj = 16 * t.tbj[c];
  const int ti = r == 0 ? i / hi : t.ti_a + (i - span_i) / hi;
  const int tj = c == 0 ? j / wj : t.tj_a + (j - span_j) / wj;
  const int li = r == 0 ? i - ti * hi : i - span_i - (ti - t.ti_a) * hi;
  const int lj = c == 0 ? j - tj * wj : j - span_j - (tj - t.tj_a) * wj;
  const float* p = a.partial + tile_first_elem(t, ti, tj) + static_cast<int64_t>(li) * wj + lj;
  const int64_t slab = slab_elems(t, r, c);
  float s = 0.f;
  for (int q = 0; q < t.ns[r][c]; ++q) s += p[q * slab];
  P[idx] = 2.0f * s;
}

// ---------------------------------------------------------------- host side
// Compiled tile families.  257-pixel patches (17 blocks a side): tiles of 9
// then 8 blocks in each direction.  129: one 9x9 tile.  65: one 5x5 tile.
// Anything else: 8x8-block tiles over the padded patch.
namespace {
struct Family {
  int i0, i1, j0, j1;
};
Family family_for(int nbi, int nbj) {
  if (nbi == 17 && nbj == 17) return {9, 8, 9, 8};
  if (nbi == 9 && nbj == 9) return {9, 9, 9, 9};
  if (nbi == 5 && nbj == 5) return {5, 5, 5, 5};
  return {8, 8, 8, 8};
}
}  // namespace

void plan_tiles(int nbi, int nbj, TilePlan* t) {
  const Family f = family_for(nbi, nbj);
  t->tbi[0] = f.i0;
  t->tbi[1] = f.i1;
  t->tbj[0] = f.j0;
  t->tbj[1] = f.j1;
  if (f.i0 != f.i1) {
    t->ti_a = 1;
    t->ti_b = 1;
  } else {
    t->ti_a = (nbi + f.i0 - 1) / f.i0;
    t->ti_b = 0;
  }
  if (f.j0 != f.j1) {
    t->tj_a = 1;
    t->tj_b = 1;
  } else {
    t->tj_a = (nbj + f.j0 - 1) / f.j0;
    t->tj_b = 0;
  }
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      t->ns[r][c] = 1;
      t->kps[r][c] = kPatchChunk;
    }
}

template <int PREC>
static hipError_t launch_family(const PatchArgs& a, dim3 grid, hipStream_t stream) {
  const TilePlan& t = a.tp;
  if (t.tbi[0] == 9 && t.tbi[1] == 8)
    hipLaunchKernelGGL((k_patch<PREC, 9, 8, 9, 8>), grid, dim3(256), 0, stream, a);
  else if (t.tbi[0] == 9)
    hipLaunchKernelGGL((k_patch<PREC, 9, 9, 9, 9>), grid, dim3(256), 0, stream, a);
  else if (t.tbi[0] == 5)
    hipLaunchKernelGGL((k_patch<PREC, 5, 5, 5, 5>), grid, dim3(256), 0, stream, a);
  else
    hipLaunchKernelGGL((k_patch<PREC, 8, 8, 8, 8>), grid, dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_patch(int prec, const PatchArgs& a, hipStream_t stream) {
  const dim3 grid(static_cast<unsigned>(tile_plan_workgroups(a.tp)));
  switch (prec) {
    case kFP32: return launch_family<kFP32>(a, grid, stream);
    case kSplitBF16: return launch_family<kSplitBF16>(a, grid, stream);
    case kSplitFP16: return launch_family<kSplitFP16>(a, grid, stream);
    case kPlainBF16: return launch_family<kPlainBF16>(a, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_finalize(const PatchArgs& a, float* P, hipStream_t stream) {
  const int64_t n = static_cast<int64_t>(a.nl) * a.nm;
  const int threads = 256;
  hipLaunchKernelGGL(k_finalize, dim3(static_cast<unsigned>((n + threads - 1) / threads)), dim3(threads), 0,
                     stream, a, P);
  return hipGetLastError();
}

}  // namespace psf
