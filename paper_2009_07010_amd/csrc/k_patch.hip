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
// A workgroup has 8 waves: 4 contraction waves and 4 generator waves, one
// of each per SIMD, so the matrix core (contraction) and the vector ALU
// (phase factors) of a SIMD work at the same time.  Per chunk of 16
// visibilities
//   * the generator waves write the next chunk's A and B columns for the
//     tile into one of two LDS buffers, in the exact operand layout of the
//     MFMA instruction (K-b), and
//   * the contraction waves run the MFMAs of the current chunk from the
//     other buffer (K-c),
// and one barrier per chunk separates writers from readers.  Each generator
// thread owns one visibility and every 8th row of A or of B: one FP64-reduced
// seed exp(2 pi i u' x_r0) and one FP64-reduced step exp(2 pi i u' 8 dl),
// then FP32 complex multiplication along the rows.
//
// Tile and wave shapes are compile-time: a tile of TBI x TBJ 16x16 blocks is
// cut into a 2 x 2 grid of contraction-wave sub-tiles whose block counts
// differ by at most one; each wave runs the loop instantiated for its own
// shape (chosen by a uniform switch on the wave index), so the contraction
// is straight-line code with no per-block conditions.
//
// Two-level accumulation: matrix-core accumulators collect a run of
// flush_chunks chunks and are then added into a second FP32 tile kept in
// LDS.  A single FP32 accumulator over a whole k-slice loses up to ~2e-5 of
// the peak at pixels where many nearly equal terms add up (the rounding of a
// long sum of similar increments is coherent); short runs keep each
// rounding small relative to the final value.
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
// group of 8 visibilities, 16 floats: 64 bytes, i.e. half of the 32 banks.
// The four 16-byte chunks of row r are stored XOR-swizzled by (r >> 1) & 3,
// which makes the 16-byte operand reads of 8 consecutive rows hit 32
// distinct banks.  A generator thread writes the rows of one residue class
// mod 8 (rows r0, r0 + 8, ...), so its swizzle is constant, and the two
// 16-lane groups of a half-wave write adjacent rows, i.e. opposite bank
// halves.
constexpr int kRowBytes = 64;
constexpr int kChunk = 16;    // visibilities per LDS chunk
constexpr int kPrefetch = 4;  // chunks of per-bin records held ahead by a generator thread

__device__ __forceinline__ int swz(int row, int chunk) { return (chunk ^ ((row >> 1) & 3)) << 4; }

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
  typedef __attribute__((address_space(3))) float lds_f32;
  typedef __attribute__((address_space(3))) uint32_t lds_u32;
  if constexpr (PREC == kFP32) {
    const int g = v >> 3, kv = v & 7;
    const int slot = (kv & 1) * 2;
    lds_t* base = hi_plane + g * gstride + row * kRowBytes + (kv >> 1) * 4;
    *reinterpret_cast<lds_f32*>(base + swz(row, slot)) = z.re;
    *reinterpret_cast<lds_f32*>(base + swz(row, slot + 1)) = z.im;
  } else {
    lds_t* p = hi_plane + row * kRowBytes + swz(row, v >> 2) + (v & 3) * 4;
    uint32_t hi, lo = 0;
    if constexpr (PREC == kSplitFP16) {
      hi = pack_f16x2(z.re, z.im);
      lo = pack_f16x2(z.re - f16_lo_to_f32(hi), z.im - f16_hi_to_f32(hi));
    } else {
      hi = pack_bf16x2(z.re, z.im);
      if constexpr (PREC == kSplitBF16) lo = pack_bf16x2(z.re - bf16_lo_to_f32(hi), z.im - bf16_hi_to_f32(hi));
    }
    *reinterpret_cast<lds_u32*>(p) = hi;
    if constexpr (PREC != kPlainBF16) *reinterpret_cast<lds_u32*>(p + lo_off) = lo;
  }
}

// LDS geometry of one tile type: two operand buffers and the second-level
// accumulator tile of the four contraction waves.
template <int PREC, int TBI, int TBJ>
struct TileGeom {
  static constexpr int TI = 16 * TBI, TJ = 16 * TBJ;
  static constexpr int RA = TI / 8, RB = TJ / 8;  // rows per generator thread (stride 8)
  static constexpr bool F32 = PREC == kFP32;
  static constexpr bool TWO = PREC == kSplitBF16 || PREC == kSplitFP16;
  static constexpr int GA = TI * kRowBytes, GB = TJ * kRowBytes;  // one group / plane
  static constexpr int APL = (F32 ? 2 : 1) * GA, BPL = (F32 ? 2 : 1) * GB;
  static constexpr int NPL = TWO ? 2 : 1;
  static constexpr int BUF = NPL * (APL + BPL);
  static constexpr int TOT = TBI * TBJ * 1024;  // per 16x16 block: 64 lanes x 4 floats
  static constexpr int LDS = 2 * BUF + TOT;
  // wave sub-tiles: rows M0 then M1 blocks, columns N0 then N1
  static constexpr int M0 = (TBI + 1) / 2, M1 = TBI / 2, N0 = (TBJ + 1) / 2, N1 = TBJ / 2;
};

// Contraction wave: sub-tile of M x N blocks at block (WI0, WJ0) of the
// tile; its second-level accumulators live in LDS at tot (block-major, in
// accumulator lane order).
template <int PREC, int TBI, int TBJ, int M, int N, int WI0, int WJ0>
__device__ __forceinline__ void mfma_wave(const PatchArgs& a, lds_t* smem, lds_t* tot, int64_t nch,
                                          float* __restrict__ out, int width) {
  using G = TileGeom<PREC, TBI, TBJ>;
  typedef __attribute__((address_space(3))) f32x4 lds_f32x4;
  typedef __attribute__((address_space(3))) bf16x8 lds_bf16x8;
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int rd = swz(lr, lg);  // swizzled chunk of this lane's operand reads (row = 16 b + lr)
  lds_f32x4* my_tot = reinterpret_cast<lds_f32x4*>(tot) + lane;

  f32x4 acc[M][N];
#pragma unroll
  for (int r = 0; r < M; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) {
      acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
      my_tot[(r * N + c) * 64] = acc[r][c];
    }
  __syncthreads();  // chunk 0 generated

  const int64_t flush = a.flush_chunks;
  for (int64_t run0 = 0; run0 < nch; run0 += flush) {
    const int64_t run1 = min(nch, run0 + flush);
    for (int64_t n = run0; n < run1; ++n) {
      const lds_t* Ah = smem + static_cast<int>(n & 1) * G::BUF;
      const lds_t* Bh = Ah + G::NPL * G::APL;
      if constexpr (G::F32) {
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          f32x4 av[M];
#pragma unroll
          for (int r = 0; r < M; ++r)
            av[r] = *reinterpret_cast<const lds_f32x4*>(Ah + g * G::GA + (16 * (WI0 + r) + lr) * kRowBytes + rd);
#pragma unroll
          for (int c = 0; c < N; ++c) {
            const f32x4 bv =
                *reinterpret_cast<const lds_f32x4*>(Bh + g * G::GB + (16 * (WJ0 + c) + lr) * kRowBytes + rd);
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
          const int off = (16 * (WI0 + r) + lr) * kRowBytes + rd;
          ah[r] = *reinterpret_cast<const lds_bf16x8*>(Ah + off);
          if constexpr (G::TWO) al[r] = *reinterpret_cast<const lds_bf16x8*>(Ah + G::APL + off);
        }
#pragma unroll
        for (int c = 0; c < N; ++c) {
          const int off = (16 * (WJ0 + c) + lr) * kRowBytes + rd;
          const bf16x8 bh = *reinterpret_cast<const lds_bf16x8*>(Bh + off);
          bf16x8 bl;
          if constexpr (G::TWO) bl = *reinterpret_cast<const lds_bf16x8*>(Bh + G::BPL + off);
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
      __syncthreads();
    }
    // second level: fold this run into the LDS tile
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
      for (int c = 0; c < N; ++c) {
        my_tot[(r * N + c) * 64] = my_tot[(r * N + c) * 64] + acc[r][c];
        acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
  }

  // partial tile of this k-slice (rows/cols beyond the patch are padding)
#pragma unroll
  for (int r = 0; r < M; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const f32x4 v = my_tot[(r * N + c) * 64];
      const int col = 16 * (WJ0 + c) + lr;  // tile-local
#pragma unroll
      for (int e = 0; e < 4; ++e) out[static_cast<size_t>(16 * (WI0 + r) + 4 * lg + e) * width + col] = v[e];
    }
}

// Generator waves: waves 4 and 5 write A (tile rows), waves 6 and 7 write B
// (tile columns).  Thread (visibility gv, class rc) of an axis writes rows
// rc, rc + 8, rc + 16, ... of that axis for every chunk: one seed at row rc
// and one step of 8 rows, both FP64-reduced.
template <int PREC, int TBI, int TBJ, bool IS_A>
__device__ __forceinline__ void gen_wave(const PatchArgs& a, lds_t* smem, int bi0, int bj0, int64_t kb,
                                         int64_t ke, int64_t nch) {
  using G = TileGeom<PREC, TBI, TBJ>;
  constexpr int R = IS_A ? G::RA : G::RB;
  const int pt = threadIdx.x - (IS_A ? 256 : 384);
  const int gv = pt & 15, rc = pt >> 4;  // rc in 0..7
  const double pos0 = IS_A ? (a.l_first + (16 * bi0 + rc) * a.dl) - a.l0 : (a.m_first + (16 * bj0 + rc) * a.dm) - a.m0;
  const double d8 = 8.0 * (IS_A ? a.dl : a.dm);
  constexpr int gstride = IS_A ? G::GA : G::GB;
  constexpr int goff = IS_A ? 0 : G::NPL * G::APL;
  constexpr int glo = IS_A ? G::APL : G::BPL;

  // Branch-free fetch (a conditional load would make the compiler wait for
  // it at once): past the end of the slice the last bin is read and its
  // weight is zeroed when used.  B needs no zeroing, A's zero weight already
  // cancels those terms.
  const double* uv_axis = reinterpret_cast<const double*>(a.uvp) + (IS_A ? 0 : 1);
  auto fetch = [&](int64_t n, double& f, cf32& cc, bool& ok) {
    const int64_t kg = kb + n * kChunk + gv;
    ok = kg < ke;
    const int64_t kc = ok ? kg : ke - 1;
    f = uv_axis[2 * kc];
    if (IS_A) {
      const float2 c = a.c[kc];
      cc = {c.x, c.y};
    }
  };
  auto generate = [&](int buf, double f, cf32 cc, bool ok) {
    cf32 z = expi_turns(f * pos0);
    cf32 zs = expi_turns(f * d8);
    if (IS_A) {
      if (!ok) cc = {0.f, 0.f};
      z = conj(cmul(cc, z));
      zs = conj(zs);
    }
    lds_t* plane = smem + buf * G::BUF + goff;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      store_operand<PREC>(plane, glo, gstride, rc + 8 * q, gv, z);
      z = cmul(z, zs);
    }
  };

  // Records are fetched kPrefetch chunks ahead into a register ring (slot =
  // chunk mod kPrefetch), which hides the latency of the global loads.
  constexpr int P = kPrefetch;
  double ring_f[P];
  cf32 ring_c[P];
  bool ring_ok[P];
  if (nch > 0) {
#pragma unroll
    for (int j = 0; j < P; ++j) fetch(j, ring_f[j], ring_c[j], ring_ok[j]);
    generate(0, ring_f[0], ring_c[0], ring_ok[0]);
    fetch(P, ring_f[0], ring_c[0], ring_ok[0]);
  }
  __syncthreads();
  // Chunk n+1 is generated while the contraction waves consume chunk n.  The
  // last iteration writes a chunk past the end (zero weights) into the idle
  // buffer; nothing reads it.
  for (int64_t n = 0; n < nch; n += P) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (n + j >= nch) break;
      const int slot = (j + 1) % P;  // holds chunk n + j + 1 (n is a multiple of P)
      generate(static_cast<int>((n + j + 1) & 1), ring_f[slot], ring_c[slot], ring_ok[slot]);
      fetch(n + j + 1 + P, ring_f[slot], ring_c[slot], ring_ok[slot]);
      __syncthreads();
    }
  }
}

template <int PREC, int TBI, int TBJ>
__device__ __forceinline__ void tile_body(const PatchArgs& a, lds_t* smem, int bi0, int bj0, int64_t kb,
                                          int64_t ke, float* out, int width) {
  using G = TileGeom<PREC, TBI, TBJ>;
  constexpr int M0 = G::M0, M1 = G::M1, N0 = G::N0, N1 = G::N1;
  const int64_t nch = ke > kb ? (ke - kb + kChunk - 1) / kChunk : 0;
  lds_t* tot = smem + 2 * G::BUF;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  switch (wave) {
    case 0: mfma_wave<PREC, TBI, TBJ, M0, N0, 0, 0>(a, smem, tot, nch, out, width); break;
    case 1: mfma_wave<PREC, TBI, TBJ, M0, N1, 0, N0>(a, smem, tot + M0 * N0 * 1024, nch, out, width); break;
    case 2: mfma_wave<PREC, TBI, TBJ, M1, N0, M0, 0>(a, smem, tot + M0 * (N0 + N1) * 1024, nch, out, width); break;
    case 3:
      mfma_wave<PREC, TBI, TBJ, M1, N1, M0, N0>(a, smem, tot + (M0 * (N0 + N1) + M1 * N0) * 1024, nch, out, width);
      break;
    case 4:
    case 5: gen_wave<PREC, TBI, TBJ, true>(a, smem, bi0, bj0, kb, ke, nch); break;
    default: gen_wave<PREC, TBI, TBJ, false>(a, smem, bi0, bj0, kb, ke, nch); break;
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
__global__ __attribute__((amdgpu_flat_work_group_size(512, 512), amdgpu_waves_per_eu(2, 2)))
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
    hipLaunchKernelGGL((k_patch<PREC, 9, 8, 9, 8>), grid, dim3(512), 0, stream, a);
  else if (t.tbi[0] == 9)
    hipLaunchKernelGGL((k_patch<PREC, 9, 9, 9, 9>), grid, dim3(512), 0, stream, a);
  else if (t.tbi[0] == 5)
    hipLaunchKernelGGL((k_patch<PREC, 5, 5, 5, 5>), grid, dim3(512), 0, stream, a);
  else
    hipLaunchKernelGGL((k_patch<PREC, 8, 8, 8, 8>), grid, dim3(512), 0, stream, a);
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
