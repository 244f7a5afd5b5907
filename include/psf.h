/*
 * psf.h -- C ABI of libpsfdecorr: position-dependent (smearing-distorted)
 * point spread functions of averaged visibilities on AMD MI355X (gfx950).
 *
 * Problem (Atemkeng et al. 2020, "Fast algorithms to approximate the
 * position-dependent point spread function responses in radio
 * interferometric wide-field imaging"):
 *
 *   Averaging visibilities over a time x frequency bin [section 2.3, the
 *   averaging integral over the sampling bin] multiplies the bin-centre
 *   visibility of a point source at (l0, m0) by a distortion factor
 *   [section 3.1, sampled distortion = bin-centre phase x distortion].
 *   Read discretely, for bin k with samples s at uvw u_s and centre u_k
 *   (wavelengths), n0 = sqrt(1 - l0^2 - m0^2):
 *
 *     phi_s = (u_s - u_k) l0 + (v_s - v_k) m0 + (w_s - w_k)(n0 - 1)
 *     D_k   = mean_s exp(-2 pi i phi_s)
 *
 *   The distorted PSF [section 2.3, distorted-PSF equation] about the
 *   source [section 2.2, offset indexing], both conjugate halves summed and
 *   the w-term linearised into u' = u - w l0/n0, v' = v - w m0/n0:
 *
 *     P_ij = 2 Re sum_k W_k D_k exp(2 pi i (u'_k x_i + v'_k y_j)),
 *     x_i = l_first + i dl - l0,   y_j = m_first + j dm - m0.
 *
 * Conventions for every entry point:
 *  - Every array pointer is a DEVICE pointer owned by the caller, except
 *    those documented as host pointers (h_*).  The library allocates no
 *    device memory and keeps no device state; scratch memory is the
 *    caller's workspace, sized with psf_workspace_bytes().
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*,
 *    NULL = the null stream), performs no host<->device synchronisation and
 *    no allocation, and clears what it needs with kernels (no memset
 *    nodes), so it may be captured into a HIP graph.  psf_autotune and
 *    psf_timing_* are the exceptions and say so.
 *  - Scalar and shape checks run on the host before anything is launched.
 *    A failed check returns PSF_EINVAL (or PSF_EWORKSPACE) and launches
 *    nothing; psf_last_error() then holds a message (thread-local).
 *    Launch failures return PSF_EDEVICE.  A device other than gfx950
 *    returns PSF_EUNSUPPORTED.  No C++ exception crosses this boundary.
 *  - Results are deterministic: partial sums are reduced in a fixed order
 *    (no floating-point atomics), so repeated calls are bitwise identical.
 */
#ifndef PSFDECORR_PSF_H
#define PSFDECORR_PSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PSF_OK = 0,
  PSF_EINVAL = -1,       /* bad argument, shape or pointer */
  PSF_EWORKSPACE = -2,   /* workspace missing or too small */
  PSF_EDEVICE = -3,      /* a HIP call or launch failed */
  PSF_EUNSUPPORTED = -4  /* current device is not gfx950 / feature absent */
} psf_status;

/* Arithmetic of the patch contraction.  Phase arguments are always formed
 * and reduced to turns in FP64; sin/cos, D_k and accumulation are FP32.
 * Accuracy of the split forms: an operand value v is carried as hi + lo
 * (16 significant bits in BF16, 22 in FP16), and one term's product is off
 * by up to 3 * 2^-16 (BF16) or 3 * 2^-22 (FP16) of |c a b|.  Over many
 * visibilities these errors are incoherent and the patch error stays far
 * below 1e-5 of the peak (measured 1e-7 to 6e-6 on the workloads of the
 * tests, the largest for 120 strongly decorrelated bins); a patch of a few
 * bins can reach the per-term bound in PSF_SPLIT_BF16 (4.6e-5 of the peak
 * at K = 1), so every entry point that contracts takes FP32 products
 * instead of split-BF16 ones when K < 256 (where they cost nothing
 * measurable). */
typedef enum {
  PSF_FP32 = 0,        /* FP32 matrix-core products, FP32 accumulation */
  PSF_SPLIT_BF16 = 1,  /* operands split hi+lo in BF16, 3 products, FP32 acc */
  PSF_SPLIT_FP16 = 2,  /* operands split hi+lo in FP16, 3 products, FP32 acc */
  PSF_PLAIN_BF16 = 3,  /* single BF16 product: a negative control, not accurate */
  PSF_MIXED_FP16 = 4,  /* see below: 2 products, for many bins */
  PSF_SR_FP16 = 5      /* see below: 1 product, for many bins */
} psf_prec;

/* PSF_MIXED_FP16: patches 65, 129 or 257 rows high (the symmetric form of
 * the contraction) with K >= 2^18 bins.  The column factors c_k b_kj are
 * split hi+lo in FP16 as in PSF_SPLIT_FP16; the row factors (cos and sin of
 * the row phase) are one FP16 value each, rounded stochastically: two
 * products instead of three.  A term is then off by up to 2^-11 of
 * |c a b|, a bound that does not keep the patch error below 1e-5 of the
 * peak by itself; the rounding is unbiased and its errors are independent
 * across bins (a bin's random word comes from its index), so the patch
 * error falls like 2^-12 sqrt(sum |c_k|^2) / |peak| (one standard
 * deviation): the largest over a 257 x 257 patch about 2e-6 of the peak at
 * 2^18 equally weighted bins with little decorrelation, and measured 5e-8 to
 * 3.3e-6 on the tests' workloads (K = 5.8M to 265M, sources to 3 deg), the
 * split forms' 7e-8 to 2.6e-6.  A patch of few effective bins (a few
 * heavily weighted bins) or whose peak is small against sum |c_k| (strong
 * decorrelation) has a larger error.  The result is deterministic: the
 * same inputs give the same bits.  Smaller K, and patches of other
 * heights, run as PSF_SPLIT_FP16; psf_patch_backward takes PSF_SPLIT_FP16
 * products for it.
 *
 * PSF_SR_FP16: as PSF_MIXED_FP16, and the column factors too are one
 * stochastically rounded FP16 value (their own random word per bin, so that
 * a term's two roundings are independent): one product per term product.
 * The same statistical bound with about 1.4 times the spread (two roundings
 * per term instead of one): measured 7e-8 to 6.3e-6 of the peak on the
 * tests' workloads (the largest on the precision workload's 2.96 deg
 * source, against a normaliser that is a lower bound of the patch's peak),
 * 6.7e-7 to 8.4e-7 over every pixel of the uniform-bin 257 x 257 PSF.  Same
 * conditions and fallbacks as PSF_MIXED_FP16. */

/* Flag OR-ed into prec for psf_patch, psf_patch_batched and
 * psf_workspace_bytes: the normalised PSF [section 4, errors taken on PSFs
 * normalised at the source; Algorithm 2, the properly normalised PSF],
 * P / peak with peak = 2 Re sum_k W_k D_k, the patch's value at the source
 * itself (every phase factor is 1 there), whether or not the grid contains
 * the source.  The peak is summed in FP64 in a fixed order from the same
 * W_k D_k the contraction uses; the division is FP64, rounded to float.
 * A peak of 0 (no visibility, or every weight 0) gives a patch of zeros.
 * Other entry points reject the flag (PSF_EINVAL). */
#define PSF_NORMALISE 0x100

/* One observation: high-resolution uvw tracks, channels and the bin table
 * (all device arrays).  Bins are ordered (baseline, time bin, frequency bin):
 * baseline b averages nt_b consecutive samples in time and nc_b consecutive
 * channels; bins tile from the first sample, the last bin along each axis
 * may be short.  Bin k = bl_koff[b] + T * ceil(n_ch / nc_b) + F. */
typedef struct psf_obs {
  int32_t n_bl;             /* baselines */
  int32_t n_t;              /* high-resolution time samples per baseline */
  int32_t n_ch;             /* channels */
  int32_t reserved;         /* must be 0 */
  int64_t K;                /* number of bins (averaged visibilities), one-sided */
  int64_t n_tb;             /* number of time bins over all baselines */
  const double* uvw_m;      /* [n_bl][n_t][3] uvw in metres */
  const double* freq_hz;    /* [n_ch] channel centre frequencies (Hz) */
  const int32_t* bl_bin;    /* [n_bl][2] {nt_b, nc_b}, both >= 1 */
  const int64_t* bl_koff;   /* [n_bl + 1] first bin of each baseline, bl_koff[n_bl] = K */
  const int64_t* bl_tboff;  /* [n_bl + 1] first time-bin row of each baseline, last = n_tb */
  const double* uvw_c_m;    /* [n_tb][3] uvw (metres) at each time-bin centre; the
                               centre frequency of a bin is the mean of its channels */
  const float* W;           /* [K] weight of each averaged visibility */
  /* Windowed averaging (section 2.3: the boxcar of the averaging integral
   * replaced by a baseline-dependent window).  Optional, NULL = boxcar on
   * that axis.  Sample (b, t, c) has weight win_t[b][t] * win_c[b][c] and
   * D_k = sum_s x_s exp(-2 pi i phi_s) / sum_s x_s over the bin's samples;
   * a bin whose window sums to 0 gets D_k = 0.  Weights must be finite (not
   * checked: device memory).  psf_decorr_sinc (Method 1) rejects windows. */
  const float* win_t;       /* [n_bl][n_t] time-window weights, or NULL */
  const float* win_c;       /* [n_bl][n_ch] channel-window weights, or NULL */
} psf_obs;

/* One source and the absolute pixel grid of its patch: pixel (i, j) is at
 * (l_first + i dl, m_first + j dm); the patch is row-major [nl][nm]
 * (i along l, j along m).  out_off is the element offset of this patch in a
 * concatenated output (P_all / G_all); psf_patch ignores it. */
typedef struct psf_src {
  double l0, m0;
  double l_first, m_first;
  double dl, dm;
  int32_t nl, nm;           /* 1 .. 4096 each */
  int64_t out_off;
} psf_src;

/* psf_patch without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same computation and kernels as psf_patch (D and
 * prec, PSF_NORMALISE included, as there), run on a scratch array of
 * 320 MiB that the library holds on every GPU it runs on until the process
 * ends.  It allocates nothing and calls no allocating routine.  Fails with
 * PSF_EWORKSPACE when the patch needs more than that scratch (its records
 * take 40 bytes per bin: about 7 million bins at 257 x 257); use
 * psf_patch with a workspace then.  The first call on a device looks up the
 * scratch address of that device (make it outside graph capture).  Every
 * call on a GPU shares that GPU's scratch: calls that overlap in time on
 * one GPU (different streams, or host threads) race and must be ordered by
 * the caller.  Nothing in the scratch needs to start at zero. */
int psf_patch_noalloc(const psf_obs* obs, const psf_src* h_src, const float* D, int prec,
                      float* P, void* stream);

/* Workspace bytes needed by psf_patch and psf_patch_fullw (n_src = 1),
 * psf_patch_batched and psf_patch_backward for these sources and precision.
 * h_srcs is a host array.  Writes the size to *out (host). */
int psf_workspace_bytes(const psf_obs* obs, int32_t n_src, const psf_src* h_srcs,
                        int prec, size_t* out);

/* D_k for every bin [section 2.3 averaging; section 3.1 bin-centre
 * factorisation], written as D[k][0] = Re, D[k][1] = Im (float, [K][2]).
 * Phases relative to the bin centre are formed in FP64 and reduced to
 * turns before FP32 sin/cos.  Needs no workspace. */
int psf_decorr(const psf_obs* obs, double l0, double m0, float* D, void* stream);

/* Method 1 of the paper, the uv-plane approximation [section 3.1]: per bin
 * the product sinc(dPsi/2) sinc(dPhi/2) of the phase changes across the
 * bin's time interval (at its centre frequency) and across its frequency
 * interval (at its centre time), 2-D (w dropped), sinc(x) = sin(x)/x.  A bin
 * of n samples spaced by s is taken to cover n s.  Only the end rows of each
 * bin are read.  Written like psf_decorr (D[k][0] = value, D[k][1] = 0), so
 * psf_patch with this D gives the Method-1 PSF.  Needs no workspace. */
int psf_decorr_sinc(const psf_obs* obs, double l0, double m0, float* D, void* stream);

/* The distorted PSF patch of one source [section 2.3, distorted-PSF
 * equation], P [nl][nm] float.  D is [K][2] from psf_decorr, or NULL to
 * compute it inside the call.  h_src is a host pointer. */
int psf_patch(const psf_obs* obs, const psf_src* h_src, const float* D, int prec,
              float* P, void* ws, size_t ws_bytes, void* stream);

/* Many sources per call [section 3.3: one PSF per source direction].
 * Sources are grouped by tile family (their patch size) and form, in groups
 * of at most 16 whose per-bin records fit 16 GiB: each source of a group
 * gets K records of 40 bytes (u', v' in FP64, the 16-pixel phase steps of
 * both axes, W D), written by one decorrelation launch per source; one
 * persistent contraction launch then runs every (source, tile, k-slice)
 * work item of the group, and one finalise launch writes its patches.  So
 * a call costs 3 launches per group, plus one per source, and its
 * workspace holds one group's records: where K is large (2.65e8 bins take
 * 10.6 GB per source) a group holds one source.  h_srcs (host) fixes sizes,
 * offsets and the plan; d_srcs (device, same n_src entries with the same
 * nl, nm, out_off) supplies directions and grids at run time, so a
 * captured graph can be replayed with new directions and grids (any grid
 * position: the plan depends on the patch sizes only).  tuning_json (host,
 * may be NULL) is a table from psf_autotune.  P_all receives every patch at
 * its out_off.  prec may carry PSF_NORMALISE. */
int psf_patch_batched(const psf_obs* obs, int32_t n_src, const psf_src* h_srcs,
                      const psf_src* d_srcs, int prec, const char* tuning_json,
                      float* P_all, void* ws, size_t ws_bytes, void* stream);

/* Adjoint of the patch with respect to the source direction, grid fixed:
 * given G_all = dLoss/dP (device, float, each source's [nl][nm] block at
 * its out_off), writes grad_lm[s][0] = dLoss/dl0, grad_lm[s][1] =
 * dLoss/dm0 (device, double, [n_src][2]).  The derivative of the patch
 * definition [section 2.3, distorted-PSF equation] runs through D_k (its
 * derivative over the bin's samples [section 2.3 averaging]), the
 * linearised w-shift u'(l0, m0), v'(l0, m0) and the pixel offsets
 * x_i = l_i - l0, y_j = m_j - m0.  For patches of up to 288 columns (rows: up to 16 ranges of row blocks whose share of
 * G fits in LDS, e.g. 2048 rows at 257 columns) it evaluates the sums per
 * visibility in reverse mode (G b and G (y b) on the matrix cores, G held
 * on chip); otherwise it
 * forms five derivative patches with the forward contraction (arithmetic
 * chosen by prec) and reduces them against G.  Both accumulate in FP64 in a
 * fixed order (deterministic).
 * h_srcs (host) gives sizes and out_off, and the directions and grids
 * when d_srcs is NULL; otherwise d_srcs (device, same entries as h_srcs)
 * supplies directions and grids at run time, so a captured forward and
 * backward can be replayed with new directions.  G_all must hold every
 * source's block: the library cannot check device extents. */
int psf_patch_backward(const psf_obs* obs, int32_t n_src, const psf_src* h_srcs,
                       const psf_src* d_srcs, const float* G_all, int prec,
                       double* grad_lm, void* ws, size_t ws_bytes, void* stream);

/* The patch with the exact w phase [section 2.1: the visibility relation
 * with its w (n - 1) term] instead of the linearised w-shift:
 *   P_ij = sum_k W_k [D_k exp(2 pi i (u_k x_i + v_k y_j + w_k (n_ij - n0))) + c.c.]
 * with n_ij = sqrt(1 - l_i^2 - m_j^2) and D_k computed (windows honoured).
 * The part of the w phase beyond its linearisation, w_k q_ij, is expanded
 * in a centred Taylor series whose terms are linearised patches with
 * modified coefficients, each contracted with the arithmetic prec; the
 * order follows from the range of q over the grid and a bound of |w| (a
 * truncation bound of 1e-7 of the coefficient sum).  *n_terms (host, may be
 * NULL) receives the number of contractions.  Fails with PSF_EINVAL when a
 * grid corner lies outside the sky or the non-linear phase spans more than
 * 4 rad over the patch (a patch too wide for the expansion).  Synchronises
 * the stream once (to read the |w| bound): not capturable.  The span check
 * needs that bound, so when it fails the factor and bound kernels have run
 * (P is not written).  ws sized with psf_workspace_bytes; P (device, float
 * [nl][nm]) must not overlap it. */
int psf_patch_fullw(const psf_obs* obs, const psf_src* h_src, int prec, float* P, int32_t* n_terms,
                    void* ws, size_t ws_bytes, void* stream);

/* Method 2, the image-plane approximation [section 3.2, Algorithm 1]: one
 * decorrelation for all baselines, pixelised over the uv plane from a
 * fringe-rate model (circular tracks turning at the sidereal rate:
 * dPsi = 2 pi omega_E (-v0 l0 + u0 m0) dt, dPhi = 2 pi (dnu/nu) |l0| |u0|,
 * D^ = sinc(dPsi/2) sinc(dPhi/2)), applied to the effective PSF (the PSF at
 * the phase centre, section 2.2) as a product of Fourier transforms.
 * Grid: N x N, N a power of two in 16..4096, square cells of `cell`
 * radians; pixel i at offset (i - N/2) cell; uv cell a at a' / (N cell)
 * wavelengths, a' = a for a < N/2 and a - N otherwise (DFT order).
 *
 * psf_method2_spectrum (once per observation and grid): the effective PSF
 * on the centred grid (patch contraction at l0 = m0 = 0, arithmetic prec,
 * windows honoured) and its forward 2-D DFT into S (device, float
 * [N][N][2], DFT order).  ws sized with psf_method2_workspace_bytes.
 *
 * psf_method2_patch (per source): P[s] = Re DFT^-1 (S D^(l0_s, m0_s)) / N^2
 * on the centred grid of offsets from the source (device, float
 * [n_src][N][N]).  h_dirs: host double [n_src][2] = (l0, m0); dt_bin and
 * dnu_bin are the averaging bin's duration (s) and bandwidth (Hz), nu the
 * frequency (Hz) of the fractional bandwidth.  Sources are processed 16 per
 * launch; ws holds min(n_src, 16) N^2 complex floats.  Neither call
 * synchronises; S must stay valid until psf_method2_patch has run. */
int psf_method2_workspace_bytes(const psf_obs* obs, int32_t N, int prec, int32_t n_src, size_t* out);
int psf_method2_spectrum(const psf_obs* obs, int32_t N, double cell, int prec, float* S, void* ws,
                         size_t ws_bytes, void* stream);
int psf_method2_patch(int32_t N, double cell, const float* S, int32_t n_src, const double* h_dirs,
                      double dt_bin, double dnu_bin, double nu, float* P, void* ws, size_t ws_bytes,
                      void* stream);

/* The flux of the patch-fitting model flux_s P_s and its adjoint, for
 * n_src sources whose patches (npix pixels each) are concatenated (device,
 * float).  psf_flux_scale: out[s][p] = flux[s] P[s][p].  psf_flux_backward:
 * given dL/dout, writes G[s][p] = flux[s] dL/dout[s][p] (float, the
 * cotangent psf_patch_backward takes) and grad_flux[s] = sum_p dL/dout[s][p]
 * P[s][p] (device double, FP64 products and sums in a fixed order).  flux is
 * a device float array [n_src].  n_src in 1..65535, npix in 1..2^31.
 * Accuracy: grad_flux is exact for the float P it is given, so its error is
 * that of P.  For the fitting loss sum ||flux P - T||^2 near its optimum the
 * terms of dL/dflux = 2 sum r P (r = flux P - T) cancel: a patch error of
 * e (relative to the patch peak) gives an error of up to e sum |2 r P| /
 * peak, which relative to the cancelled sum itself is measured at up to
 * 1.6e-4 with split-BF16 patches and 8e-5 with FP32 patches on the
 * differentiation workload (16 sources of 129^2, K = 5.8M; below 1e-5 of
 * sum |2 r P| everywhere). */
int psf_flux_scale(int32_t n_src, int64_t npix, const float* flux, const float* P, float* out, void* stream);
int psf_flux_backward(int32_t n_src, int64_t npix, const float* flux, const float* P, const float* grad_out,
                      float* G, double* grad_flux, void* stream);

/* Hogbom CLEAN with position-dependent PSFs [Algorithm 2]: up to max_iter
 * minor cycles on the image `residual` (device, float [nl][nm] on the grid
 * of h_grid, whose l0, m0 are ignored; in: the dirty image, out: the
 * residual).  Each cycle takes the peak pixel of |residual| (the first
 * maximum in row-major order), evaluates the distorted PSF of that
 * direction on the image grid with the arithmetic prec (as psf_patch,
 * decorrelation factors computed), subtracts gain * peak * PSF / PSF(peak)
 * and records the component (pixel comp_i, comp_j, amplitude gain * peak;
 * host arrays of max_iter entries; *n_comp receives the count).  Stops
 * early when |peak| < threshold; an observation without visibilities
 * (K = 0, a zero PSF) runs no cycle; a peak pixel off the sky fails with
 * PSF_EINVAL.  gain in (0, 1].  Synchronises the stream once per cycle to
 * read the peak: not capturable (psf_clean_hogbom_device is).  ws sized with
 * psf_clean_workspace_bytes. */
int psf_clean_workspace_bytes(const psf_obs* obs, const psf_src* h_grid, int prec, size_t* out);
int psf_clean_hogbom(const psf_obs* obs, const psf_src* h_grid, float* residual, int32_t max_iter, double gain,
                     double threshold, int prec, int32_t* comp_i, int32_t* comp_j, float* comp_amp,
                     int32_t* n_comp, void* ws, size_t ws_bytes, void* stream);

/* Hogbom CLEAN with position-dependent PSFs [Algorithm 2], kept on the
 * device so that it can be captured into a graph and replayed: as
 * psf_clean_hogbom, but the peak is placed by a kernel (the PSF's direction
 * goes to a source record in the workspace that the decorrelation and the
 * contraction read when they run), the stream is never synchronised, and
 * exactly n_iter cycles are launched.  Once |peak| falls below threshold (or
 * is 0, or its pixel lies off the sky) cleaning stops: the remaining cycles
 * still evaluate a PSF but subtract nothing.  comp_i, comp_j, comp_amp
 * (n_iter entries) and *n_comp are DEVICE memory; *n_comp is written before
 * the first cycle.  For the same inputs the residual and the components
 * equal those of psf_clean_hogbom bit for bit (which instead fails with
 * PSF_EINVAL at a peak off the sky).  Same workspace as
 * psf_clean_hogbom (psf_clean_workspace_bytes); the call allocates nothing. */
int psf_clean_hogbom_device(const psf_obs* obs, const psf_src* h_grid, float* residual, int32_t n_iter, double gain,
                            double threshold, int prec, int32_t* comp_i, int32_t* comp_j, float* comp_amp,
                            int32_t* n_comp, void* ws, size_t ws_bytes, void* stream);

/* Hogbom CLEAN with Method-2 PSFs [Algorithm 2 with the section 3.2
 * approximation]: as psf_clean_hogbom, but the PSF of each peak's direction
 * is the Method-2 patch (psf_method2_patch from the spectrum S of
 * psf_method2_spectrum, N x N at the image's cell, which must be square),
 * laid with its centre (offset 0, index N/2) on the peak pixel; image
 * pixels beyond its extent are not changed.  dt_bin, dnu_bin, nu as for
 * psf_method2_patch.  Synchronises the stream once per cycle: not
 * capturable.  ws sized with psf_clean_method2_workspace_bytes. */
int psf_clean_method2_workspace_bytes(int32_t N, const psf_src* h_grid, size_t* out);
int psf_clean_hogbom_method2(int32_t N, const float* S, const psf_src* h_grid, float* residual, int32_t max_iter,
                             double gain, double threshold, double dt_bin, double dnu_bin, double nu,
                             int32_t* comp_i, int32_t* comp_j, float* comp_amp, int32_t* n_comp, void* ws,
                             size_t ws_bytes, void* stream);

/* Hogbom CLEAN with Method-2 PSFs [Algorithm 2 with the section 3.2
 * approximation], kept on the device as psf_clean_hogbom_device is for
 * exact PSFs: the peak is placed by a kernel, the Method-2 patch reads its
 * direction from device memory, exactly n_iter cycles are launched (those
 * past the threshold subtract nothing), no synchronisation, so the loop can
 * be captured into a graph.  comp_i, comp_j, comp_amp (n_iter entries) and
 * *n_comp are DEVICE memory.  For the same inputs the residual and the
 * components equal those of psf_clean_hogbom_method2 bit for bit.  ws sized
 * with psf_clean_method2_workspace_bytes; the call allocates nothing. */
int psf_clean_hogbom_method2_device(int32_t N, const float* S, const psf_src* h_grid, float* residual,
                                    int32_t n_iter, double gain, double threshold, double dt_bin, double dnu_bin,
                                    double nu, int32_t* comp_i, int32_t* comp_j, float* comp_amp, int32_t* n_comp,
                                    void* ws, size_t ws_bytes, void* stream);

/* Times candidate launch shapes for these sources with HIP events and
 * writes a JSON tuning table (host buffer json_out, capacity json_cap).
 * Synchronises the stream: not capturable. */
int psf_autotune(const psf_obs* obs, int32_t n_src, const psf_src* h_srcs, int prec,
                 void* ws, size_t ws_bytes, char* json_out, size_t json_cap, void* stream);

/* Optional timing of the contraction kernels: while enabled, every launch
 * of a patch or adjoint contraction is bracketed by HIP events on its
 * stream.  psf_timing_read synchronises and returns the summed kernel time
 * (ms) and the number of launches since the last read.  Not capturable. */
int psf_timing_enable(int on);
int psf_timing_read(double* ms_total, int64_t* launches);

const char* psf_strerror(int status);
const char* psf_last_error(void);
/* Library version string. */
const char* psf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PSFDECORR_PSF_H */
