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
// A workgroup has 8 waves, two per SIMD.  Every wave both contracts and
// generates: per chunk of 16 visibilities it
//   * runs the MFMAs of its sub-tile of the output tile on the current
//     chunk's A and B columns from one of two LDS buffers (K-c), and,
//     interleaved with those MFMAs in the same instruction stream,
//   * writes its share of the next chunk's A or B columns into the other
//     buffer, in the exact operand layout of the MFMA instruction (K-b),
// and one barrier per chunk separates writers from readers.  Interleaving
// lets the vector ALU work of the phase factors issue while the matrix core
// executes.  Waves 0-3 generate A (tile rows), waves 4-7 B (tile columns),
// so each SIMD holds one of each: a generating thread owns one visibility
// and every 16th row, with one FP64-reduced seed and one FP64-reduced step
// of 16 rows, then an FP32 recurrence along the rows.
//
// Tile and wave shapes are compile-time: a tile of TBI x TBJ 16x16 blocks is
// cut into eight sub-tiles (wave_shape); each wave runs the loop
// instantiated for its own shape and axis (chosen by a uniform switch on the
// wave index), so the contraction is straight-line code with no per-block
// conditions.
//
// Two-level accumulation: matrix-core accumulators collect a run of
// flush_chunks chunks and are then added into a second FP32 tile, the
// workgroup's own partial slab in global memory (read-modify-write, no
// atomics; it stays cache-resident).  A single FP32 accumulator over a whole k-slice loses up to ~2e-5 of
// the peak at pixels where many nearly equal terms add up (the rounding of a
// long sum of similar increments is coherent); short runs keep each
// rounding small relative to the final value.
//
// Split forms: every operand value v is stored as hi = round16(v) and
// lo = round16(v - hi); the product uses hi*hi + hi*lo + lo*hi (three MFMAs)
// with FP32 accumulation.
//
// Mixed form (symmetric form only): the columns c_k b_kj are split as above,
// the rows (cos and sin) are one FP16 value each: a * (b_hi + b_lo), two
// MFMAs.  Rounded to nearest, a row value would carry an error that
// neighbouring visibilities share (their phases are nearly equal, and where
// the phase is small cos rounds to 1 for all of them), which adds up
// coherently over a baseline's bins.  The rows are instead rounded
// stochastically (the conversion instruction's random-word operand, a
// per-visibility Weyl sequence in the bin index): unbiased, with errors
// independent across visibilities, which average out over many of them.
// Stochastic form (symmetric form only): the columns too are one
// stochastically rounded FP16 value (their own per-visibility random word,
// a hash of the bin index, so that a term's two roundings are independent):
// a * b, one MFMA.
//
// Symmetric form.  With N = 2h + 1 rows, x_i = delta + (i - h) dl where
// delta = (l_first + h dl) - l0 is the offset of the grid's centre row from
// the source (0 for a centred grid), so a_ki = e_k a_k(s_i) with
// e_k = exp(2 pi i u'_k delta) and s_i = (i - h) dl symmetric about 0;
// a_k(-s) = conj(a_k(s)), so with C = Re a and S = Im a (even and odd in s)
// and d_kj = c_k e_k b_kj,
//   P(+-s, y_j) = 2 sum_k [C_k(s) Re d_kj -+ S_k(s) Im d_kj],   s >= 0.
// The contraction then runs over an inner dimension of K real values
// (instead of 2K) into an output of h + 1 "C" rows (x = 0 .. h, against
// Re d) and h "S" rows (x = 1 .. h, against Im d): half the multiply-adds
// of the general form, for the same (2h + 1) x N output.  C rows sit at
// output rows x + 15 of the first CB blocks, S rows at 16 CB + x - 1 of the
// blocks after (h a multiple of 16, CB = h/16 + 1), so a generating thread
// with row class rc walks one phase sequence x = rc - 15 + 16 n and writes
// its cosine to C row block n and its sine to S row block CB + n - 1.
// Rows 0..14 (x < 0) are never read.  B columns carry c_k b_kj, its real
// part in one LDS plane and its imaginary part in another; a contraction
// wave's rows lie in one group and read the matching plane.  K-f combines
// the C and S rows of |x| into the rows +x and -x.
#include <type_traits>

#include "psf_device.hpp"
#include "psf_kernels.hpp"

namespace psf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
// LDS byte pointer (address space 3), so that every operand access is a
// ds_read / ds_write with a 32-bit address rather than a flat access.
typedef __attribute__((address_space(3))) uint8_t lds_t;

// One LDS operand row: 32 16-bit values (16 visibilities x re/im) or, per
// group of 8 visibilities, 16 floats: 64 bytes, i.e. half of the 32 banks.
// The four 16-byte chunks of row r are stored XOR-swizzled by (r >> 1) & 3,
// which makes the 16-byte operand reads of 8 consecutive rows hit 32
// distinct banks.  A generating thread writes the rows of one residue class
// mod 16 (rows r0, r0 + 16, ...), so its swizzle is constant, and the 16-lane
// groups of a wave write adjacent rows.
constexpr int kRowBytes = 64;
constexpr int kChunk = 16;    // visibilities per LDS chunk

__device__ __forceinline__ int swz(int row, int chunk) { return (chunk ^ ((row >> 1) & 3)) << 4; }

// What the tile body needs of one work item's source.
struct TileArgs {
  const BinRec* rec;
  const float2* c;
  double l_first, dl, l0, m_first, dm, m0;
  // symmetric form: offset of the grid's centre row from the source,
  // (l_first + h dl) - l0 (0 for a grid centred on the source)
  double delta_l;
  int flush_chunks;
};

template <int PREC>
__device__ __forceinline__ f32x4 mfma16(const bf16x8& a, const bf16x8& b, f32x4 acc) {
  if constexpr (PREC == kSplitFP16 || PREC == kMixedFP16 || PREC == kSRFP16) {
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
    // lo = v - hi, exact in FP32 (hi widened back: a shift or a mask for
    // BF16, a conversion for FP16)
    uint32_t hi, lo = 0;
    if constexpr (PREC == kSplitFP16) {
      hi = pack_f16x2(z.re, z.im);
      lo = f16_lo_pair(hi, z.re, z.im);
    } else {
      hi = pack_bf16x2(z.re, z.im);
      if constexpr (PREC == kSplitBF16) lo = pack_bf16x2(z.re - bf16_lo_to_f32(hi), z.im - bf16_hi_to_f32(hi));
    }
    *reinterpret_cast<lds_u32*>(p) = hi;
    if constexpr (PREC != kPlainBF16) *reinterpret_cast<lds_u32*>(p + lo_off) = lo;
  }
}

// Leading C blocks (rows of the symmetric form's C group) of each tile
// type of the symmetric families: 257 rows (tiles of 9 C blocks and 8 S
// blocks), 129 (one tile, 5 + 4), 65 (one tile, 3 + 2); -1 otherwise.
__host__ __device__ constexpr int sym_cb(int TBI, int TBJ) {
  return (TBJ == 17 && TBI == 9) ? 9
         : (TBJ == 17 && TBI == 8) ? 0
         : (TBI == 9 && TBJ == 9)  ? 5
         : (TBI == 5 && TBJ == 5)  ? 3
                                   : -1;
}

// LDS geometry of one tile type: two operand buffers.
template <int PREC, int TBI, int TBJ, bool SYM = false>
struct TileGeom {
  static constexpr int TI = 16 * TBI, TJ = 16 * TBJ;
  static constexpr int RA = TI / 8, RB = TJ / 8;  // rows per generator thread (stride 8)
  static constexpr bool F32 = PREC == kFP32;
  // operands carried as hi + lo (A: tile rows, B: tile columns)
  static constexpr bool TWOA = PREC == kSplitBF16 || PREC == kSplitFP16;
  static constexpr bool TWOB = TWOA || PREC == kMixedFP16;
  static constexpr int GA = TI * kRowBytes, GB = TJ * kRowBytes;  // one group / plane
  static constexpr int APL = (F32 ? 2 : 1) * GA, BPL = (F32 ? 2 : 1) * GB;
  static constexpr int NPLA = TWOA ? 2 : 1, NPLB = TWOB ? 2 : 1;
  // symmetric form: C blocks of the tile, and B planes (Re d and Im d when
  // the tile holds both groups, else the one its rows read)
  static constexpr int CB = SYM ? sym_cb(TBI, TBJ) : TBI;
  static constexpr int NBP = SYM && CB > 0 && CB < TBI ? 2 : 1;
  static constexpr int BUF = NPLA * APL + NBP * NPLB * BPL;
  // byte offset of B's part (0 hi, 1 lo) of plane pl within a buffer
  static constexpr int boff(int part, int pl) { return NPLA * APL + (pl * NPLB + part) * BPL; }
  // Chunk buffers.  2: the chunk being contracted and the chunk being
  // generated.  3: also the next chunk, complete one barrier early, so that
  // its first operand fragments can be read ahead of the barrier (measured
  // slower on the 257-pixel tiles, kept selectable).
  static constexpr int NBUF = 2;
  static constexpr int LDS = NBUF * BUF;
  static_assert(LDS <= 160 * 1024, "LDS of a workgroup exceeds 160 KiB");
  static_assert(!SYM || CB >= 0, "no symmetric form for this tile type");
  static_assert(SYM || (PREC != kMixedFP16 && PREC != kSRFP16),
                "the mixed and stochastic forms exist for the symmetric form only");
};

// Sub-tile of one contraction wave: m x n blocks at block (i0, j0) of the
// tile; bit (r n + c) of `mask` set where block (i0 + r, j0 + c) belongs to
// the wave.  Waves w and w + 4 share SIMD w mod 4.
struct WaveShape {
  int m, n, i0, j0;
  uint64_t mask;
};
__host__ __device__ constexpr uint64_t full_mask(int m, int n) { return m * n == 64 ? ~0ULL : (1ULL << (m * n)) - 1; }

__host__ __device__ constexpr WaveShape wave_shape(int TBI, int TBJ, int w, bool sym = false) {
  // Symmetric 9 x 9 tile: waves 0-3 take the 5 C block rows, waves 4-7 the
  // 4 S block rows (a wave's rows must lie in one group), columns split so
  // that the busiest SIMD has 22 blocks (5 a + 4 b per SIMD: 21, 22, 19, 19).
  if (sym && TBI == 9 && TBJ == 9) {
    const int a[4] = {1, 2, 3, 3};
    const int b[4] = {4, 3, 1, 1};
    const int s = w & 3;
    int j0 = 0;
    for (int q = 0; q < s; ++q) j0 += w < 4 ? a[q] : b[q];
    const int m = w < 4 ? 5 : 4, n = w < 4 ? a[s] : b[s];
    return {m, n, w < 4 ? 0 : 5, j0, full_mask(m, n)};
  }
  if (TBI == 9 && TBJ == 17) {
    // 153 blocks, at most 20 per wave: four 5x4 sub-tiles over rows 0-4 and
    // columns 0-15, three 4x5 over rows 5-8 and columns 0-14, and the rest
    // (column 16, and column 15 of rows 5-8) as a 9x2 sub-tile with its
    // top-left 5x1 strip masked out.
    if (w < 4) return {5, 4, 0, 4 * w, full_mask(5, 4)};
    if (w < 7) return {4, 5, 5, 5 * (w - 4), full_mask(4, 5)};
    uint64_t m = full_mask(9, 2);
    for (int r = 0; r < 5; ++r) m &= ~(1ULL << (2 * r));
    return {9, 2, 0, 15, m};
  }
  // 9 x 9: two block-row groups of 3 and 6 rows; wave s (s < 4) takes
  // columns a[s] of the first, wave 4 + s columns b[s] of the second, which
  // gives at most 21 blocks per SIMD (waves s and 4 + s share a SIMD; found
  // by exhaustive search) against 23 for the default cut.
  if (TBI == 9 && TBJ == 9) {
    const int r0 = 3;
    const int a[4] = {1, 2, 3, 3};
    const int b[4] = {3, 2, 2, 2};
    const int s = w & 3;
    int j0 = 0;
    for (int q = 0; q < s; ++q) j0 += w < 4 ? a[q] : b[q];
    const int m = w < 4 ? r0 : TBI - r0, n = w < 4 ? a[s] : b[s];
    return {m, n, w < 4 ? 0 : r0, j0, full_mask(m, n)};
  }
  // Otherwise 2 block-row groups x 4 block-column groups whose sizes differ
  // by at most one; the second row group takes the column groups shifted by
  // one, so every SIMD gets one larger and one smaller sub-tile.
  const int m0 = (TBI + 1) / 2;
  const int q = w < 4 ? w : (w - 3) % 4;
  const int j0 = (TBJ * q) / 4, n = (TBJ * (q + 1)) / 4 - j0;
  return w < 4 ? WaveShape{m0, n, 0, j0, full_mask(m0, n)}
               : WaveShape{TBI - m0, n, m0, j0, full_mask(TBI - m0, n)};
}

// A 16-byte vector store reads its data registers after it issues; a VALU
// write to those registers in the very next cycle can change what is stored
// (seen as corrupted slab elements when the compiler placed a 64-bit move
// into the stored registers right after the store).  One wait state after
// each slab store closes that window.
__device__ __forceinline__ void store_data_guard() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 1");
  __builtin_amdgcn_sched_barrier(0);
}

// True if the eight contraction-wave sub-tiles cover every block of the tile
// exactly once and no sub-tile holds more than 30 blocks (120 accumulator
// registers).
template <int TBI, int TBJ, bool SYM = false>
constexpr bool wave_shapes_ok() {
  int cover[TBI * TBJ] = {};
  for (int w = 0; w < 8; ++w) {
    const WaveShape s = wave_shape(TBI, TBJ, w, SYM);
    if (s.m * s.n > 64 || s.i0 + s.m > TBI || s.j0 + s.n > TBJ) return false;
    // symmetric form: a wave's rows lie in one group (C or S)
    if (SYM && !(s.i0 + s.m <= sym_cb(TBI, TBJ) || s.i0 >= sym_cb(TBI, TBJ))) return false;
    int nb = 0;
    for (int r = 0; r < s.m; ++r)
      for (int c = 0; c < s.n; ++c)
        if ((s.mask >> (r * s.n + c)) & 1) {
          ++cover[(s.i0 + r) * TBJ + s.j0 + c];
          ++nb;
        }
    if (nb > 30) return false;
  }
  for (int b = 0; b < TBI * TBJ; ++b)
    if (cover[b] != 1) return false;
  return true;
}

// Phase-factor generation of one wave (K-b).  Waves 0-3 write A (tile rows),
// waves 4-7 write B (tile columns), so each SIMD (waves w and w + 4) holds
// one of each.  Thread (visibility gv, class rc = 4 (w mod 4) + lane / 16)
// writes rows rc, rc + 16, ... of its axis for every chunk: one FP64-reduced
// seed at row rc (hardware sine and cosine: used once, its 4e-7 error stays
// far below the split's rounding) and the bin's 16-row step (formed once per bin with the
// records), then along the rows: for the split forms the real three-term
// recurrence z+ = 2 cos(t) z - z- of a unit step e^{it} (two fused
// multiply-adds per row instead of a complex product).  Its error grows
// with the row count and with the conditioning of the rounded 2 cos(t) near
// small steps: at most 1.3e-5 of an element over 17 rows (a step near 1e-3
// rad), against 9e-7 for the complex product and about 8e-6 for the split
// representation itself; across visibilities these errors are incoherent,
// and the patch errors are unchanged.  The FP32 form, the precision
// baseline, keeps the complex product.  A row class is constant mod 8, so the thread's
// swizzle is constant.  Per-bin records are fetched one chunk ahead:
// deeper prefetch rings measured slower, their register shifts costing more
// vector issue slots than the latency they hide.
template <int PREC, int TBI, int TBJ, bool IS_A>
struct Gen {
  using G = TileGeom<PREC, TBI, TBJ>;
  static constexpr int R = IS_A ? TBI : TBJ;  // rows per thread
  static constexpr int GSTRIDE = IS_A ? G::GA : G::GB;
  static constexpr int GOFF = IS_A ? 0 : G::NPLA * G::APL;
  static constexpr int GLO = IS_A ? G::APL : G::BPL;
  static constexpr int P = 1;  // chunks of records held ahead

  int gv, rc;
  double pos0;
  const BinRec* recs;
  const float2* cptr;
  int64_t kb, ke;
  double rf[P];   // u' (A) or v' (B)
  cf32 rst[P];    // 16-row step
  cf32 rcc[P];    // W D (A)
  bool rok[P];
  cf32 z, zp;  // current and previous row's factor (zp: the step itself in FP32)
  float tc;    // 2 cos t of the 16-row step (split forms)
  lds_t* plane;

  __device__ __forceinline__ Gen(const TileArgs& a, int wave, int bi0, int bj0, int64_t kb_, int64_t ke_) {
    const int lane = threadIdx.x & 63;
    gv = lane & 15;
    rc = 4 * (wave & 3) + (lane >> 4);
    pos0 = IS_A ? (a.l_first + (16 * bi0 + rc) * a.dl) - a.l0 : (a.m_first + (16 * bj0 + rc) * a.dm) - a.m0;
    recs = a.rec;
    cptr = a.c;
    kb = kb_;
    ke = ke_;
  }
  // Branch-free fetch (a conditional load would make the compiler wait for
  // it at once): past the end of the slice the last bin is read and its
  // weight is zeroed when used.  B needs no zeroing, A's zero weight already
  // cancels those terms.
  __device__ __forceinline__ void fetch(int64_t n, double& f, cf32& st, cf32& cc, bool& ok) const {
    const int64_t kg = kb + n * kChunk + gv;
    ok = kg < ke;
    const int64_t kc = ok ? kg : ke - 1;
    const BinRec* r = recs + kc;
    f = IS_A ? r->up : r->vp;
    const float2 s = IS_A ? r->step_a : r->step_b;
    st = {s.x, s.y};
    if (IS_A) {
      const float2 c = cptr[kc];
      cc = {c.x, c.y};
    }
  }
  __device__ __forceinline__ void prime() {
#pragma unroll
    for (int j = 0; j < P; ++j) fetch(j, rf[j], rst[j], rcc[j], rok[j]);
  }
  // Seed and step of the chunk held in ring slot 0, to be written into
  // buffer buf (the step comes with the record).
  __device__ __forceinline__ void begin(lds_t* smem, int buf) {
    z = expi_turns_hw(rf[0] * pos0);  // the seed is used once: hardware sin/cos
    cf32 zs = rst[0];
    if (IS_A) {
      const cf32 cc = rok[0] ? rcc[0] : cf32{0.f, 0.f};
      z = conj(cmul(cc, z));
      zs = conj(zs);
    }
    if constexpr (PREC == kFP32) {
      zp = zs;
    } else {
      zp = cmul(z, conj(zs));  // the row before the seed
      tc = 2.0f * zs.re;
    }
    plane = smem + buf * G::BUF + GOFF;
  }
  // Rows [q0, q1) of the current chunk (q0, q1 fold to constants once the
  // caller's loops are unrolled).
  __device__ __forceinline__ void rows(int q0, int q1) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (q < q0 || q >= q1) continue;
      store_operand<PREC>(plane, GLO, GSTRIDE, rc + 16 * q, gv, z);
      if constexpr (PREC == kFP32) {
        z = cmul(z, zp);
      } else {
        const cf32 zn = {__builtin_fmaf(tc, z.re, -zp.re), __builtin_fmaf(tc, z.im, -zp.im)};
        zp = z;
        z = zn;
      }
    }
  }
  // Shift the ring by one chunk and fetch chunk n into its last slot.
  __device__ __forceinline__ void advance(int64_t n) {
#pragma unroll
    for (int j = 0; j + 1 < P; ++j) {
      rf[j] = rf[j + 1];
      rst[j] = rst[j + 1];
      rcc[j] = rcc[j + 1];
      rok[j] = rok[j + 1];
    }
    fetch(n, rf[P - 1], rst[P - 1], rcc[P - 1], rok[P - 1]);
  }
};

// Store two real operand values of visibilities 2 gv and 2 gv + 1 (of the
// 32 of a symmetric-form chunk) at `row` of a plane.  16-bit: k index
// within the row = visibility, one 32-bit store of the packed pair (hi),
// one of lo.  FP32: two groups of 16 visibilities (group stride gstride),
// within a group visibility 4 c + e at float e of 16-byte chunk c (lane
// group c of the 16x16x4 instruction takes chunk c, k-step e float e), so
// the pair is one 8-byte store.
template <int PREC>
__device__ __forceinline__ void store_pair(lds_t* hi_plane, int lo_off, int gstride, int row, int gv, float v0,
                                           float v1) {
  typedef __attribute__((address_space(3))) uint64_t lds_u64;
  typedef __attribute__((address_space(3))) uint32_t lds_u32;
  if constexpr (PREC == kFP32) {
    lds_t* p = hi_plane + (gv >> 3) * gstride + row * kRowBytes + swz(row, (gv & 7) >> 1) + (gv & 1) * 8;
    // the pair as one 64-bit word, v0 in the low half (a two-float vector
    // store here had the compiler build the pair through scratch memory)
    *reinterpret_cast<lds_u64*>(p) = (static_cast<uint64_t>(__builtin_bit_cast(uint32_t, v1)) << 32) |
                                     __builtin_bit_cast(uint32_t, v0);
  } else {
    lds_t* p = hi_plane + row * kRowBytes + swz(row, gv >> 2) + (gv & 3) * 4;
    uint32_t hi, lo = 0;
    if constexpr (PREC == kSplitFP16) {
      hi = pack_f16x2(v0, v1);
      lo = f16_lo_pair(hi, v0, v1);
    } else {
      hi = pack_bf16x2(v0, v1);
      if constexpr (PREC == kSplitBF16) lo = pack_bf16x2(v0 - bf16_lo_to_f32(hi), v1 - bf16_hi_to_f32(hi));
    }
    *reinterpret_cast<lds_u32*>(p) = hi;
    if constexpr (PREC != kPlainBF16) *reinterpret_cast<lds_u32*>(p + lo_off) = lo;
  }
}

// Mixed form: two row values of visibilities 2 gv and 2 gv + 1 (random
// words r0, r1) as one FP16 value each, rounded stochastically: the
// conversion adds the top bits of the random word below the kept ones and
// truncates, so each value rounds up with probability equal to its
// fractional position between its two FP16 neighbours.
__device__ __forceinline__ void store_pair_sr(lds_t* plane, int row, int gv, float v0, float v1, uint32_t r0,
                                              uint32_t r1) {
  typedef __attribute__((address_space(3))) uint32_t lds_u32;
  // each conversion writes one half and keeps the other; the two together
  // write both, so the initial value is never read (left undefined, so that
  // no register is cleared for it)
  f16x2_t h;
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wuninitialized"
  h = __builtin_amdgcn_cvt_sr_f16_f32(h, v0, r0, false);
#pragma clang diagnostic pop
  h = __builtin_amdgcn_cvt_sr_f16_f32(h, v1, r1, true);
  *reinterpret_cast<lds_u32*>(plane + row * kRowBytes + swz(row, gv >> 2) + (gv & 3) * 4) =
      __builtin_bit_cast(uint32_t, h);
}

// Phase-factor generation of the symmetric form (see the file comment).
// Thread (gv, rc) owns visibilities 2 gv and 2 gv + 1 of each 32-visibility
// chunk and row (column) class rc.  A (waves 0-3): unit n of its sequence
// is x = (rc - 15 + 16 n) dl; it writes Re a to C row 16 n + rc (n < CB)
// and Im a to S row 16 (CB + n - 1) + rc (n >= 1).  B (waves 4-7): unit q
// is column 16 q + rc, y its offset from m0; it writes Re and/or Im of
// d = c b to the tile's B plane(s).  Seeds are FP64-reduced and evaluated
// once (hardware sine and cosine), the 16-row steps come with the bin's
// record; along the units the split forms use the real three-term
// recurrence (one fused multiply-add per written value; both parts when
// both are written), the FP32 form the complex product.  Past the end of
// the slice the records and coefficients read as 0 (see fetch), so the
// coefficient (carried by B) is 0.
template <int PREC, int TBI, int TBJ, bool IS_A>
struct GenSym {
  using G = TileGeom<PREC, TBI, TBJ, true>;
  // how this side's values are stored: stochastically rounded (store_pair_sr)
  // for the rows of the mixed form and both sides of the stochastic form,
  // else split or FP32 (store_pair<OP>)
  static constexpr int OP = PREC == kMixedFP16 ? kSplitFP16 : PREC;
  static constexpr bool SR = (IS_A && PREC == kMixedFP16) || PREC == kSRFP16;
  static constexpr int CB = G::CB;
  static constexpr bool HC = CB > 0, HS = CB < TBI;
  static constexpr int N0 = IS_A && !HC ? 1 : 0;
  static constexpr int NA = (HC ? CB - 1 : 0) > (HS ? TBI - CB : 0) ? (HC ? CB - 1 : 0) : (HS ? TBI - CB : 0);
  static constexpr int R = IS_A ? NA - N0 + 1 : TBJ;  // generator units per chunk
  // which parts of the factor are written: both, or only the imaginary one
  static constexpr bool BOTH = IS_A ? (HC && HS) : G::NBP == 2;
  static constexpr bool ONLY_IM = !BOTH && (IS_A ? !HC : CB == 0);
  static constexpr int GSTRIDE = IS_A ? G::GA : G::GB;
  static constexpr int LO = IS_A ? G::APL : G::BPL;
  static constexpr int P = 1;  // chunks of records held ahead

  int gv, rc;
  double pos0;
  const BinRec* recs;
  const float2* cptr;
  int64_t kb, ke;
  double delta;  // B: the grid centre's offset from the source along l
  double rf[P][2];
  double ru[P][2];  // B: u' (for the offset factor)
  cf32 rst[P][2];
  cf32 rcc[P][2];
  bool rok[P][2];      // pointer form: the bin lies inside the slice
  uint32_t rrw[P][2];  // stochastic rounding: the bins' random words
  uint32_t rw[2];
  uint32_t wl;  // A, stochastic rounding: this thread's part of the rows' word
  int vo, vc;   // byte offsets of this thread's first bin in a chunk's records and coefficients
  cf32 z[2], zp[2];
  float tc[2];
  lds_t* plane;

  __device__ __forceinline__ GenSym(const TileArgs& a, int wave, int bi0, int bj0, int64_t kb_, int64_t ke_) {
    (void)bi0;
    const int lane = threadIdx.x & 63;
    gv = lane & 15;
    rc = 4 * (wave & 3) + (lane >> 4);
    pos0 = IS_A ? static_cast<double>(rc - 15 + 16 * N0) * a.dl : (a.m_first + (16 * bj0 + rc) * a.dm) - a.m0;
    delta = a.delta_l;
    recs = a.rec;
    cptr = a.c;
    kb = kb_;
    ke = ke_;
    vo = 2 * gv * static_cast<int>(sizeof(BinRec));
    vc = 2 * gv * static_cast<int>(sizeof(float2));
    if (BUF && PREC != kSRFP16) asm volatile("" : "+v"(vo), "+v"(vc));
    if (BUF && SR && IS_A) {
      wl = static_cast<uint32_t>(2 * gv) * kWeyl;
      // kept opaque, so that the compiler does not fold the per-chunk sum
      // below back into one product per bin
      asm volatile("" : "+v"(wl));
    }
  }
  static constexpr uint32_t kWeyl = 0x9E3779B1u;
  // How a chunk's records and coefficients are read (same values either
  // way).  Buffer form: through buffer resources that start at the chunk's
  // first bin and end at the slice's end (ke), so bins past it read as 0
  // (u' = v' = 0, a zero step and c = 0: their B values are 0, no
  // contribution, and their A values finite); the resources are uniform
  // (scalar) and a thread's offsets into them fixed, so no per-bin address
  // arithmetic remains (65- and 129-pixel stochastic families 4-7% faster).
  // Pointer form, kept for the B waves of the 257-pixel stochastic tiles:
  // that kernel sits at the 128-register limit of four waves per SIMD,
  // where the buffer form on both sides made the allocator spill inside the
  // chunk loop (9% slower); past the slice's end it reads the last bin and
  // takes c = 0.
  static constexpr bool BUF = !(PREC == kSRFP16 && TBJ >= 17 && !IS_A);
  // The random word of bin kg: for the rows kg times the golden ratio mod
  // 2^32, whose top bits (the ones the conversion uses) are equidistributed
  // in kg; for the columns a 32-bit mixing hash of kg (multiply-xorshift
  // finaliser), independent of the rows' word.
  static __device__ __forceinline__ uint32_t col_word(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
  }
  // Bin kg = k0 + 2 gv + e of chunk n (k0 = kb + 32 n).
  // The thread's offsets for one chunk, kept opaque to the compiler so that
  // the per-bin and per-field constants added to them become the load
  // instructions' immediate offsets rather than one register per load: in
  // the stochastic form a fresh copy per chunk, which the compiler cannot
  // hoist out of the chunk loop either (its four waves per SIMD leave no
  // registers for hoisted offsets: 1-2% faster), elsewhere the offsets made
  // opaque once (a copy per chunk was 2% slower for the two-wave 257-pixel
  // split kernel).
  __device__ __forceinline__ int2 offsets() const {
    int2 v = {vo, vc};
    if (BUF && PREC == kSRFP16) asm volatile("" : "+v"(v.x), "+v"(v.y));
    return v;
  }
  __device__ __forceinline__ void fetch(int64_t n, int e, int2 vof, double& f, double& u, cf32& st, cf32& cc,
                                        bool& ok, uint32_t& rwd) const {
    const int64_t k0 = kb + n * kPatchChunkSym;
    const int j = 2 * gv + e;
    if constexpr (!BUF) {
      const int64_t kg = k0 + j;
      if (SR) rwd = IS_A ? static_cast<uint32_t>(kg) * kWeyl : col_word(static_cast<uint32_t>(kg));
      ok = kg < ke;
      const int64_t kc = ok ? kg : ke - 1;
      const BinRec* r = recs + kc;
      f = IS_A ? r->up : r->vp;
      const float2 s = IS_A ? r->step_a : r->step_b;
      st = {s.x, s.y};
      if (!IS_A) {
        u = r->up;
        const float2 c = cptr[kc];
        cc = {c.x, c.y};
      }
      return;
    }
    // the rows' word as (k0 + e) times the multiplier (uniform) plus this
    // thread's part
    if (SR) rwd = IS_A ? static_cast<uint32_t>(k0 + e) * kWeyl + wl : col_word(static_cast<uint32_t>(k0 + j));
    const int64_t left = ke - k0;
    const int nb = left <= 0 ? 0 : left >= kPatchChunkSym ? kPatchChunkSym : static_cast<int>(left);
    const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<BinRec*>(recs + k0), 0, nb * static_cast<int>(sizeof(BinRec)), 0x00020000);
    const int ro = vof.x + e * static_cast<int>(sizeof(BinRec));
    if (IS_A) {
      f = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rr, ro + offsetof(BinRec, up), 0, 0));
      st = __builtin_bit_cast(cf32, __builtin_amdgcn_raw_buffer_load_b64(rr, ro + offsetof(BinRec, step_a), 0, 0));
    } else {
      const u32x4_t uv = __builtin_amdgcn_raw_buffer_load_b128(rr, ro + offsetof(BinRec, up), 0, 0);
      u = __builtin_bit_cast(double, __builtin_shufflevector(uv, uv, 0, 1));
      f = __builtin_bit_cast(double, __builtin_shufflevector(uv, uv, 2, 3));
      st = __builtin_bit_cast(cf32, __builtin_amdgcn_raw_buffer_load_b64(rr, ro + offsetof(BinRec, step_b), 0, 0));
      const __amdgpu_buffer_rsrc_t rcs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float2*>(cptr + k0), 0, nb * static_cast<int>(sizeof(float2)), 0x00020000);
      cc = __builtin_bit_cast(cf32,
                              __builtin_amdgcn_raw_buffer_load_b64(rcs, vof.y + e * static_cast<int>(sizeof(float2)), 0, 0));
    }
  }
  __device__ __forceinline__ void prime() {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int2 vof = offsets();
#pragma unroll
      for (int e = 0; e < 2; ++e) fetch(j, e, vof, rf[j][e], ru[j][e], rst[j][e], rcc[j][e], rok[j][e], rrw[j][e]);
    }
  }
  __device__ __forceinline__ void begin(lds_t* smem, int buf) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (SR) rw[e] = rrw[0][e];
      z[e] = expi_turns_hw(rf[0][e] * pos0);
      const cf32 zs = rst[0][e];
      if (!IS_A) {
        cf32 cc = BUF || rok[0][e] ? rcc[0][e] : cf32{0.f, 0.f};
        // a grid not centred on the source: the row-independent factor
        // exp(2 pi i u' delta) joins the coefficient (FP64-reduced, used once)
        if (delta != 0.0) cc = cmul(cc, expi_turns_hw(ru[0][e] * delta));
        z[e] = cmul(cc, z[e]);
      }
      if constexpr (PREC == kFP32) {
        zp[e] = zs;
      } else {
        zp[e] = cmul(z[e], conj(zs));  // the unit before the seed
        tc[e] = 2.0f * zs.re;
      }
    }
    plane = smem + buf * G::BUF + (IS_A ? 0 : G::boff(0, 0));
  }
  __device__ __forceinline__ void step() {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if constexpr (PREC == kFP32) {
        z[e] = cmul(z[e], zp[e]);
      } else {
        cf32 zn = z[e];
        if (BOTH || !ONLY_IM) zn.re = __builtin_fmaf(tc[e], z[e].re, -zp[e].re);
        if (BOTH || ONLY_IM) zn.im = __builtin_fmaf(tc[e], z[e].im, -zp[e].im);
        zp[e] = z[e];
        z[e] = zn;
      }
    }
  }
  // Units [q0, q1) of the current chunk.
  __device__ __forceinline__ void rows(int q0, int q1) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (q < q0 || q >= q1) continue;
      if constexpr (SR && !IS_A) {
        if constexpr (BOTH) {
          store_pair_sr(plane, 16 * q + rc, gv, z[0].re, z[1].re, rw[0], rw[1]);
          store_pair_sr(plane + G::NPLB * G::BPL, 16 * q + rc, gv, z[0].im, z[1].im, rw[0], rw[1]);
        } else if constexpr (ONLY_IM) {
          store_pair_sr(plane, 16 * q + rc, gv, z[0].im, z[1].im, rw[0], rw[1]);
        } else {
          store_pair_sr(plane, 16 * q + rc, gv, z[0].re, z[1].re, rw[0], rw[1]);
        }
      } else if constexpr (SR) {
        const int n = N0 + q;
        if (HC && n < CB) store_pair_sr(plane, 16 * n + rc, gv, z[0].re, z[1].re, rw[0], rw[1]);
        if (HS && n >= 1 && CB + n - 1 < TBI)
          store_pair_sr(plane, 16 * (CB + n - 1) + rc, gv, z[0].im, z[1].im, rw[0], rw[1]);
      } else if constexpr (IS_A) {
        const int n = N0 + q;
        if (HC && n < CB) store_pair<OP>(plane, LO, GSTRIDE, 16 * n + rc, gv, z[0].re, z[1].re);
        if (HS && n >= 1 && CB + n - 1 < TBI)
          store_pair<OP>(plane, LO, GSTRIDE, 16 * (CB + n - 1) + rc, gv, z[0].im, z[1].im);
      } else {
        if constexpr (BOTH) {
          store_pair<OP>(plane, LO, GSTRIDE, 16 * q + rc, gv, z[0].re, z[1].re);
          store_pair<OP>(plane + G::NPLB * G::BPL, LO, GSTRIDE, 16 * q + rc, gv, z[0].im, z[1].im);
        } else if constexpr (ONLY_IM) {
          store_pair<OP>(plane, LO, GSTRIDE, 16 * q + rc, gv, z[0].im, z[1].im);
        } else {
          store_pair<OP>(plane, LO, GSTRIDE, 16 * q + rc, gv, z[0].re, z[1].re);
        }
      }
      if (q + 1 < R) step();
    }
  }
  __device__ __forceinline__ void advance(int64_t n) {
#pragma unroll
    for (int j = 0; j + 1 < P; ++j)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        rf[j][e] = rf[j + 1][e];
        ru[j][e] = ru[j + 1][e];
        rst[j][e] = rst[j + 1][e];
        rcc[j][e] = rcc[j + 1][e];
        rok[j][e] = rok[j + 1][e];
        rrw[j][e] = rrw[j + 1][e];
      }
    const int2 vof = offsets();
#pragma unroll
    for (int e = 0; e < 2; ++e)
      fetch(n, e, vof, rf[P - 1][e], ru[P - 1][e], rst[P - 1][e], rcc[P - 1][e], rok[P - 1][e], rrw[P - 1][e]);
  }
};

// One wave on one work item: the contraction of its sub-tile (K-c) for
// chunk n, interleaved with the generation of its rows of chunk n + 1 into
// the other LDS buffer, then one barrier.  Its second-level accumulators
// are its blocks of the workgroup's partial slab in global memory, laid out
// [block][lane][4] in accumulator lane order (block = tile row block * TBJ +
// tile column block).
template <int PREC, int TBI, int TBJ, int W, bool SYM = false>
__device__ __forceinline__ void wave_item(const TileArgs& a, lds_t* smem, int bi0, int bj0, int64_t kb, int64_t ke,
                                          float* __restrict__ slab) {
  static_assert(wave_shapes_ok<TBI, TBJ, SYM>(), "contraction waves must cover the tile once");
  using G = TileGeom<PREC, TBI, TBJ, SYM>;
  constexpr WaveShape S = wave_shape(TBI, TBJ, W, SYM);
  constexpr int M = S.m, N = S.n, WI0 = S.i0, WJ0 = S.j0;
  constexpr auto on = [](int r, int c) { return ((S.mask >> (r * N + c)) & 1) != 0; };
  constexpr bool IS_A = W < 4;
  using Gn = std::conditional_t<SYM, GenSym<PREC, TBI, TBJ, IS_A>, Gen<PREC, TBI, TBJ, IS_A>>;
  constexpr int R = Gn::R;
  // visibilities per chunk, and the B plane this wave's rows read (the
  // symmetric form's S rows read Im d when the tile holds both groups)
  constexpr int CH = SYM ? kPatchChunkSym : kChunk;
  constexpr int BP = G::NBP == 2 && WI0 >= G::CB ? 1 : 0;
  // generation rows spread over the contraction steps of a chunk (the
  // mixed and stochastic forms have no second pass)
  constexpr int NSTEP = G::F32 ? 2 * N : PREC == kMixedFP16 || PREC == kSRFP16 ? N : N + M;
  typedef __attribute__((address_space(3))) f32x4 lds_f32x4;
  typedef __attribute__((address_space(3))) bf16x8 lds_bf16x8;
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int rd = swz(lr, lg);  // swizzled chunk of this lane's operand reads (row = 16 b + lr)
  // The slab is reached through a buffer resource: the lane offset is the
  // only per-lane address register and each block's offset is a scalar, so
  // no 64-bit block addresses are held across the contraction loop.
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(slab, 0, 256 * TBI * TBJ * static_cast<int>(sizeof(float)), 0x00020000);
  const int voff = lane * 16;
  auto slab_ld = [&](int blk) {
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, blk * 1024, 0));
  };
  auto slab_st = [&](int blk, f32x4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), rs, voff, blk * 1024, 0);
    store_data_guard();
  };

  const int64_t nch = ke > kb ? (ke - kb + CH - 1) / CH : 0;
  Gn gen(a, W, bi0, bj0, kb, ke);
  // With NBUF chunk buffers, chunks 0 .. NBUF - 2 are generated before the
  // loop; in the loop, chunk n is contracted from buffer n mod NBUF while
  // chunk n + NBUF - 1 is generated into buffer (n + NBUF - 1) mod NBUF.
  // With three buffers the first operand fragments of chunk n + 1 (complete
  // since the previous barrier) are read ahead of the barrier.
  constexpr int NB = G::NBUF;
  if (nch > 0) {
    gen.prime();
#pragma unroll
    for (int b = 0; b + 1 < NB; ++b) {
      gen.begin(smem, b);
      gen.rows(0, R);
      gen.advance(Gn::P + b);
    }
  }
  f32x4 acc[M][N];
#pragma unroll
  for (int r = 0; r < M; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  __syncthreads();  // the first NBUF - 1 chunks generated

  auto buf_at = [&](int b) { return static_cast<const lds_t*>(smem + b * G::BUF); };
  auto ldA = [&](const lds_t* Ah, int plane, int r) {
    return *reinterpret_cast<const lds_bf16x8*>(Ah + plane * G::APL + (16 * (WI0 + r) + lr) * kRowBytes + rd);
  };
  auto ldB = [&](const lds_t* Ah, int plane, int c) {
    return *reinterpret_cast<const lds_bf16x8*>(Ah + G::boff(plane, BP) + (16 * (WJ0 + c) + lr) * kRowBytes + rd);
  };
  auto ldA32 = [&](const lds_t* Ah, int g, int r) {
    return *reinterpret_cast<const lds_f32x4*>(Ah + g * G::GA + (16 * (WI0 + r) + lr) * kRowBytes + rd);
  };
  // first operand fragments of the chunk about to be contracted
  bf16x8 pah[M], pbh = {}, pbl = {};
  f32x4 pav[M];
  auto prefetch = [&](const lds_t* Ah) {
    if constexpr (G::F32) {
#pragma unroll
      for (int r = 0; r < M; ++r) pav[r] = ldA32(Ah, 0, r);
    } else {
#pragma unroll
      for (int r = 0; r < M; ++r) pah[r] = ldA(Ah, 0, r);
      pbh = ldB(Ah, 0, 0);
      if constexpr (G::TWOB) pbl = ldB(Ah, 1, 0);
    }
  };
  int cur = 0;  // buffer of chunk n
  if (NB == 3 && nch > 0) prefetch(buf_at(0));

  const int64_t flush = a.flush_chunks;
  for (int64_t run0 = 0; run0 < nch; run0 += flush) {
    const int64_t run1 = min(nch, run0 + flush);
    for (int64_t n = run0; n < run1; ++n) {
      const int nxt = cur + 1 == NB ? 0 : cur + 1;
      const int gen_buf = NB == 2 ? nxt : (nxt + 1 == NB ? 0 : nxt + 1);
      const lds_t* Ah = buf_at(cur);
      const lds_t* Bh = Ah + G::boff(0, BP);
      if (NB == 2) prefetch(Ah);
      // Chunk n + NBUF - 1 (past the end near the last chunk: zero weights,
      // written into an idle buffer and never read).
      gen.begin(smem, gen_buf);
      int step = 0;
      auto gen_step = [&]() {
        gen.rows((step * R) / NSTEP, ((step + 1) * R) / NSTEP);
        ++step;
        __builtin_amdgcn_sched_barrier(0);
      };
      if constexpr (G::F32) {
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          f32x4 av[M];
#pragma unroll
          for (int r = 0; r < M; ++r) av[r] = g == 0 ? pav[r] : ldA32(Ah, g, r);
#pragma unroll
          for (int c = 0; c < N; ++c) {
            const f32x4 bv =
                *reinterpret_cast<const lds_f32x4*>(Bh + g * G::GB + (16 * (WJ0 + c) + lr) * kRowBytes + rd);
#pragma unroll
            for (int r = 0; r < M; ++r)
              if (on(r, c))
#pragma unroll
                for (int e = 0; e < 4; ++e)
                  acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r][e], bv[e], acc[r][c], 0, 0, 0);
            gen_step();
          }
        }
      } else {
        // pass 1: A_hi x (B_hi, B_lo), keeping every B_hi fragment;
        // pass 2 (split forms): A_lo x B_hi.  Loads run one column (pass 1)
        // or one row (pass 2) ahead of their MFMAs.
        bf16x8 bh[N];
        bf16x8 nbh = pbh, nbl = pbl;
#pragma unroll
        for (int c = 0; c < N; ++c) {
          bh[c] = nbh;
          const bf16x8 bl = nbl;
          if (c + 1 < N) {
            nbh = ldB(Ah, 0, c + 1);
            if constexpr (G::TWOB) nbl = ldB(Ah, 1, c + 1);
          }
#pragma unroll
          for (int r = 0; r < M; ++r) {
            if (!on(r, c)) continue;
            acc[r][c] = mfma16<PREC>(pah[r], bh[c], acc[r][c]);
            if constexpr (G::TWOB) acc[r][c] = mfma16<PREC>(pah[r], bl, acc[r][c]);
          }
          gen_step();
        }
        if constexpr (G::TWOA) {
          bf16x8 nal = ldA(Ah, 1, 0);
#pragma unroll
          for (int r = 0; r < M; ++r) {
            const bf16x8 al = nal;
            if (r + 1 < M) nal = ldA(Ah, 1, r + 1);
#pragma unroll
            for (int c = 0; c < N; ++c)
              if (on(r, c)) acc[r][c] = mfma16<PREC>(al, bh[c], acc[r][c]);
            gen_step();
          }
        } else if constexpr (PREC != kMixedFP16 && PREC != kSRFP16) {
#pragma unroll
          for (int r = 0; r < M; ++r) gen_step();
        }
      }
      gen.advance(n + (NB - 1) + Gn::P);
      if (NB == 3 && n + 1 < nch) prefetch(buf_at(nxt));
      cur = nxt;
      __syncthreads();
    }
    // second level: fold this run into the slab (the first run initialises
    // it), one block row at a time so that the loaded partials do not all
    // need registers at once
    const bool first = run0 == 0;
#pragma unroll
    for (int r = 0; r < M; ++r) {
#pragma unroll
      for (int c = 0; c < N; ++c) {
        if (!on(r, c)) continue;
        const int blk = (WI0 + r) * TBJ + (WJ0 + c);
        slab_st(blk, first ? acc[r][c] : slab_ld(blk) + acc[r][c]);
        acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if (nch == 0) {
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
      for (int c = 0; c < N; ++c)
        if (on(r, c)) slab_st((WI0 + r) * TBJ + (WJ0 + c), acc[r][c]);
  }
}

// ---------------------------------------------------------------- tile plan
// Templates over the plan's type so that device code indexes a plan in the
// kernel-argument segment in place (constant address space, scalar loads).
template <class TP>
__host__ __device__ inline int64_t slab_elems(const TP& t, int r, int c) {
  return 256LL * t.tbi[r] * t.tbj[c];
}
template <class TP>
__host__ __device__ inline int64_t row_wgs(const TP& t, int r) {
  return static_cast<int64_t>(t.tj_a) * t.ns[r][0] + static_cast<int64_t>(t.tj_b) * t.ns[r][1];
}
template <class TP>
__host__ __device__ inline int64_t row_elems(const TP& t, int r) {
  return static_cast<int64_t>(t.tj_a) * t.ns[r][0] * slab_elems(t, r, 0) +
         static_cast<int64_t>(t.tj_b) * t.ns[r][1] * slab_elems(t, r, 1);
}
// Element offset of the first slab of tile (ti, tj).
template <class TP>
__host__ __device__ inline int64_t tile_first_elem(const TP& t, int ti, int tj) {
  const int r = ti < t.ti_a ? 0 : 1;
  const int ra = ti < t.ti_a ? ti : t.ti_a, rb = ti - ra;
  const int ca = tj < t.tj_a ? tj : t.tj_a, cb = tj - ca;
  return ra * row_elems(t, 0) + rb * row_elems(t, 1) + ca * t.ns[r][0] * slab_elems(t, r, 0) +
         cb * t.ns[r][1] * slab_elems(t, r, 1);
}

int tile_max_simd_blocks(int tbi, int tbj, bool sym) {
  int mx = 0;
  for (int q = 0; q < 4; ++q) {
    int nb = 0;
    for (int w = q; w < 8; w += 4) nb += __builtin_popcountll(wave_shape(tbi, tbj, w, sym).mask);
    mx = nb > mx ? nb : mx;
  }
  return mx;
}

int64_t tile_plan_items(const TilePlan& t) {
  return t.ti_a * row_wgs(t, 0) + t.ti_b * row_wgs(t, 1);
}
size_t tile_plan_partial_elems(const TilePlan& t) {
  return static_cast<size_t>(t.ti_a * row_elems(t, 0) + t.ti_b * row_elems(t, 1));
}

typedef const __attribute__((address_space(4))) SrcPlan karg_plan;

// One work item, decoded.
struct Item {
  int type;  // tile type: row type * 2 + column type
  int bi0, bj0;
  int64_t kb, ke;
  float* slab;
  TileArgs ta;
};

__device__ __forceinline__ Item decode_item(const BatchArgs& a, karg_plan* plans, int64_t item) {
  int s = 0;
  while (s + 1 < a.n_src && item >= plans[s + 1].item0) ++s;
  karg_plan& p = plans[s];
  const auto& t = p.tp;
  // (tile row, tile column, k-slice) from the item index
  int64_t w = item - p.item0;
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
  Item it;
  it.type = r * 2 + c;
  it.bi0 = ti < t.ti_a ? ti * t.tbi[0] : t.ti_a * t.tbi[0] + (ti - t.ti_a) * t.tbi[1];
  it.bj0 = tj < t.tj_a ? tj * t.tbj[0] : t.tj_a * t.tbj[0] + (tj - t.tj_a) * t.tbj[1];
  const int64_t kps = t.kps[r][c];
  it.kb = static_cast<int64_t>(split) * kps;
  it.ke = min(a.K, it.kb + kps);
  it.slab = p.partial + tile_first_elem(t, ti, tj) + static_cast<int64_t>(split) * slab_elems(t, r, c);
  it.ta.rec = p.rec;
  it.ta.c = p.c;
  it.ta.flush_chunks = a.flush_chunks;
  if (p.dir != nullptr) {
    it.ta.l0 = p.dir[0];
    it.ta.m0 = p.dir[1];
    it.ta.l_first = p.dir[2];
    it.ta.m_first = p.dir[3];
    it.ta.dl = p.dir[4];
    it.ta.dm = p.dir[5];
  } else {
    it.ta.l0 = p.l0;
    it.ta.m0 = p.m0;
    it.ta.l_first = p.l_first;
    it.ta.m_first = p.m_first;
    it.ta.dl = p.dl;
    it.ta.dm = p.dm;
  }
  it.ta.delta_l = (it.ta.l_first + ((p.nl - 1) / 2) * it.ta.dl) - it.ta.l0;
  return it;
}

// The persistent item loop of one wave role.  Every wave of a workgroup
// takes the same items, so the barriers inside the items match; the last
// barrier of an item orders its LDS reads before the next item's first LDS
// writes.  Each role has its own loop so that what the compiler keeps live
// across items is only that role's.
template <int PREC, int I0, int I1, int J0, int J1, int ROLE, bool SYM>
__device__ __forceinline__ void role_loop(const BatchArgs& a, karg_plan* plans, lds_t* smem) {
  for (int64_t item = blockIdx.x; item < a.n_items; item += gridDim.x) {
    const Item it = decode_item(a, plans, item);
    switch (it.type) {
      case 0: wave_item<PREC, I0, J0, ROLE, SYM>(it.ta, smem, it.bi0, it.bj0, it.kb, it.ke, it.slab); break;
      case 1: wave_item<PREC, I0, J1, ROLE, SYM>(it.ta, smem, it.bi0, it.bj0, it.kb, it.ke, it.slab); break;
      case 2: wave_item<PREC, I1, J0, ROLE, SYM>(it.ta, smem, it.bi0, it.bj0, it.kb, it.ke, it.slab); break;
      default: wave_item<PREC, I1, J1, ROLE, SYM>(it.ta, smem, it.bi0, it.bj0, it.kb, it.ke, it.slab); break;
    }
  }
}

// The contraction kernel: a persistent loop over the work items of the
// launch's sources.  Template arguments are the two tile heights and the two
// tile widths (in blocks) of its tile family, and the form (general or
// symmetric) of every source of the launch.
// Waves per SIMD: two (one workgroup per compute unit) for the large tiles,
// whose registers and LDS fill a CU; four (two workgroups) for the 5 x 5
// block tiles of the 65-pixel family, whose per-chunk matrix work is small
// enough that a second workgroup's waves are needed to cover the barrier and
// LDS latency of each chunk (16 patches of 65 pixels at K = 23.2M,
// split-BF16: 38.0 to 28.6 ms), and four for every tile of the stochastic
// form, whose one product per block leaves each chunk mostly latency
// (single 257 x 257 patch at K = 5.8M: 1.58 to 1.27 ms, though the
// compiler keeps 128 registers by spilling some of the item-loop state;
// 16 patches of 129: 11.8 to 8.7 ms).
template <int PREC, int I0, int I1, int J0, int J1, bool SYM>
__global__ __attribute__((amdgpu_flat_work_group_size(512, 512),
                          amdgpu_waves_per_eu(PREC == kSRFP16 ? 4 : 2, I0 <= 5 || PREC == kSRFP16 ? 4 : 2)))
void k_patch(BatchArgs a) {
  constexpr int L00 = TileGeom<PREC, I0, J0, SYM>::LDS, L01 = TileGeom<PREC, I0, J1, SYM>::LDS;
  constexpr int L10 = TileGeom<PREC, I1, J0, SYM>::LDS, L11 = TileGeom<PREC, I1, J1, SYM>::LDS;
  constexpr int LA = L00 > L01 ? L00 : L01, LB = L10 > L11 ? L10 : L11;
  __shared__ __attribute__((aligned(16))) uint8_t smem_raw[LA > LB ? LA : LB];
  lds_t* smem = (lds_t*)smem_raw;
  // The per-source plans are read straight from the kernel-argument segment
  // (the argument starts at its offset 0): indexing the by-value parameter
  // with a run-time index would copy it to private memory.
  typedef const __attribute__((address_space(4))) uint8_t karg_byte;
  karg_plan* plans = (karg_plan*)((karg_byte*)__builtin_amdgcn_kernarg_segment_ptr() + offsetof(BatchArgs, src));
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  switch (wave) {
    case 0: role_loop<PREC, I0, I1, J0, J1, 0, SYM>(a, plans, smem); break;
    case 1: role_loop<PREC, I0, I1, J0, J1, 1, SYM>(a, plans, smem); break;
    case 2: role_loop<PREC, I0, I1, J0, J1, 2, SYM>(a, plans, smem); break;
    case 3: role_loop<PREC, I0, I1, J0, J1, 3, SYM>(a, plans, smem); break;
    case 4: role_loop<PREC, I0, I1, J0, J1, 4, SYM>(a, plans, smem); break;
    case 5: role_loop<PREC, I0, I1, J0, J1, 5, SYM>(a, plans, smem); break;
    case 6: role_loop<PREC, I0, I1, J0, J1, 6, SYM>(a, plans, smem); break;
    default: role_loop<PREC, I0, I1, J0, J1, 7, SYM>(a, plans, smem); break;
  }
}

// Sum over the k-slices of one element (row i, column j of the
// contraction's output) of a source's partial slabs, in slice order.
__device__ __forceinline__ float slab_sum(karg_plan& p, int i, int j) {
  const auto& t = p.tp;
  const int span_i = t.ti_a * 16 * t.tbi[0], span_j = t.tj_a * 16 * t.tbj[0];
  const int r = i < span_i ? 0 : 1, c = j < span_j ? 0 : 1;
  const int hi = 16 * t.tbi[r], wj = 16 * t.tbj[c];  // tile height and width in pixels
  const int ti = r == 0 ? i / hi : t.ti_a + (i - span_i) / hi;
  const int tj = c == 0 ? j / wj : t.tj_a + (j - span_j) / wj;
  const int li = r == 0 ? i - ti * hi : i - span_i - (ti - t.ti_a) * hi;
  const int lj = c == 0 ? j - tj * wj : j - span_j - (tj - t.tj_a) * wj;
  // slab layout [block][lane][4]: block (li/16, lj/16), lane = col + 16 (row/4), element row % 4
  const int blk = (li >> 4) * t.tbj[c] + (lj >> 4);
  const int rr = li & 15, cc = lj & 15;
  const float* q = p.partial + tile_first_elem(t, ti, tj) + (static_cast<int64_t>(blk) * 64 + cc + 16 * (rr >> 2)) * 4 +
                   (rr & 3);
  const int64_t slab = slab_elems(t, r, c);
  // slices added in order; 16 loads are issued before their adds so that
  // their latencies overlap (same sum, bit for bit)
  const int nsl = t.ns[r][c];
  float sum = 0.f;
  int n = 0;
  for (; n + 16 <= nsl; n += 16) {
    float v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = q[(n + u) * slab];
#pragma unroll
    for (int u = 0; u < 16; ++u) sum += v[u];
  }
  for (; n < nsl; ++n) sum += q[n * slab];
  return sum;
}

// a6: P / peak, FP64 division; 0 where the peak is 0 (no visibility or
// every weight 0: the normalised PSF is undefined).
__device__ __forceinline__ float normalised(float v, double peak) {
  return peak != 0.0 ? static_cast<float>(static_cast<double>(v) / peak) : 0.0f;
}

// K-f: P = 2 * sum over the k-slices of the pixel's tile, in slice order.
// Grid row y is source y of the launch.
__global__ __launch_bounds__(256) void k_finalize(BatchArgs a) {
  (void)a;
  typedef const __attribute__((address_space(4))) uint8_t karg_byte;
  karg_plan& p = ((karg_plan*)((karg_byte*)__builtin_amdgcn_kernarg_segment_ptr() + offsetof(BatchArgs, src)))[blockIdx.y];
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(p.nl) * p.nm) return;
  const int i = static_cast<int>(idx / p.nm), j = static_cast<int>(idx - static_cast<int64_t>(i) * p.nm);
  if (p.sym) {
    // symmetric form: row i has offset s = i - h from the grid's centre row;
    // C row |s| + 15 and S row 16 CB + |s| - 1 of the contraction give
    // P(+-|s|) = 2 (C -+ S)
    const int h = (p.nl - 1) / 2, cb = h / 16 + 1;
    const int s = i - h, as = s < 0 ? -s : s;
    const float c = slab_sum(p, as + 15, j);
    const float sn = as > 0 ? slab_sum(p, 16 * cb + as - 1, j) : 0.f;
    const float v = 2.0f * (s >= 0 ? c - sn : c + sn);
    p.P[idx] = p.peak == nullptr ? v : normalised(v, *p.peak);
    return;
  }
  const float v = 2.0f * slab_sum(p, i, j);
  p.P[idx] = p.peak == nullptr ? v : normalised(v, *p.peak);
}

// a6: one block per range of K; FP64 sum of Re c in a fixed order
__global__ __launch_bounds__(256) void k_peak_partial(const float2* __restrict__ c, int64_t K,
                                                      double* __restrict__ part) {
  const int64_t span = (K + kPeakBlocks - 1) / kPeakBlocks;
  const int64_t k0 = blockIdx.x * span, k1 = min(K, k0 + span);
  double acc = 0.0;
  for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) acc += static_cast<double>(c[k].x);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ double w[4];
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((w[0] + w[1]) + w[2]) + w[3];
}

__global__ __launch_bounds__(64) void k_peak_final(const double* __restrict__ part, double* __restrict__ peak) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < kPeakBlocks; b += 64) acc += part[b];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (threadIdx.x == 0) *peak = 2.0 * acc;
}

hipError_t launch_peak(const float2* c, int64_t K, double* scratch, double* peak, hipStream_t stream) {
  hipLaunchKernelGGL(k_peak_partial, dim3(kPeakBlocks), dim3(256), 0, stream, c, K, scratch);
  hipLaunchKernelGGL(k_peak_final, dim3(1), dim3(64), 0, stream, scratch, peak);
  return hipGetLastError();
}

// ---------------------------------------------------------------- host side
// Compiled tile families.  257-pixel patches (17 blocks a side): full-width
// tiles of 9 then 8 block rows.  129: one 9x9 tile.  65: one 5x5 tile.
// Anything else: 8x8-block tiles over the padded patch.
namespace {
struct Family {
  int i0, i1, j0, j1;
};
Family family_for(int nbi, int nbj) {
  if (nbi == 17 && nbj == 17) return {9, 8, 17, 17};
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

int tile_wgs_per_cu(const TilePlan& t, int prec) { return t.tbi[0] <= 5 || prec == kSRFP16 ? 2 : 1; }

bool sym_patch_size(int nl, int nm) {
  const int nbj = (nm + 15) / 16;
  return (nl == 257 && nbj == 17) || (nl == 129 && nbj == 9) || (nl == 65 && nbj == 5);
}

template <int PREC>
static hipError_t launch_family(const BatchArgs& a, dim3 grid, hipStream_t stream) {
  const TilePlan& t = a.src[0].tp;
  if (a.src[0].sym) {
    if (t.tbi[0] == 9 && t.tbi[1] == 8)
      hipLaunchKernelGGL((k_patch<PREC, 9, 8, 17, 17, true>), grid, dim3(512), 0, stream, a);
    else if (t.tbi[0] == 9)
      hipLaunchKernelGGL((k_patch<PREC, 9, 9, 9, 9, true>), grid, dim3(512), 0, stream, a);
    else if (t.tbi[0] == 5)
      hipLaunchKernelGGL((k_patch<PREC, 5, 5, 5, 5, true>), grid, dim3(512), 0, stream, a);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if constexpr (PREC == kMixedFP16 || PREC == kSRFP16) {
    return hipErrorInvalidValue;  // symmetric form only
  } else {
    if (t.tbi[0] == 9 && t.tbi[1] == 8)
      hipLaunchKernelGGL((k_patch<PREC, 9, 8, 17, 17, false>), grid, dim3(512), 0, stream, a);
    else if (t.tbi[0] == 9)
      hipLaunchKernelGGL((k_patch<PREC, 9, 9, 9, 9, false>), grid, dim3(512), 0, stream, a);
    else if (t.tbi[0] == 5)
      hipLaunchKernelGGL((k_patch<PREC, 5, 5, 5, 5, false>), grid, dim3(512), 0, stream, a);
    else
      hipLaunchKernelGGL((k_patch<PREC, 8, 8, 8, 8, false>), grid, dim3(512), 0, stream, a);
    return hipGetLastError();
  }
}

hipError_t launch_patch(int prec, const BatchArgs& a, int64_t n_wg, hipStream_t stream) {
  if (a.n_src < 1 || a.n_src > kMaxBatch || n_wg < 1) return hipErrorInvalidValue;
  for (int s = 1; s < a.n_src; ++s)  // one tile family and one form per launch
    if (a.src[s].tp.tbi[0] != a.src[0].tp.tbi[0] || a.src[s].tp.tbi[1] != a.src[0].tp.tbi[1] ||
        a.src[s].tp.tbj[0] != a.src[0].tp.tbj[0] || a.src[s].tp.tbj[1] != a.src[0].tp.tbj[1] ||
        a.src[s].sym != a.src[0].sym)
      return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(n_wg));
  switch (prec) {
    case kFP32: return launch_family<kFP32>(a, grid, stream);
    case kSplitBF16: return launch_family<kSplitBF16>(a, grid, stream);
    case kSplitFP16: return launch_family<kSplitFP16>(a, grid, stream);
    case kPlainBF16: return launch_family<kPlainBF16>(a, grid, stream);
    case kMixedFP16: return launch_family<kMixedFP16>(a, grid, stream);
    case kSRFP16: return launch_family<kSRFP16>(a, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_finalize(const BatchArgs& a, hipStream_t stream) {
  int64_t n = 0;
  for (int s = 0; s < a.n_src; ++s) n = max(n, static_cast<int64_t>(a.src[s].nl) * a.src[s].nm);
  const int threads = 256;
  hipLaunchKernelGGL(k_finalize, dim3(static_cast<unsigned>((n + threads - 1) / threads), a.n_src),
                     dim3(threads), 0, stream, a);
  return hipGetLastError();
}

}  // namespace psf
