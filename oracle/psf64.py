"""Plain FP64 evaluation of the distorted PSF of averaged visibilities.

TEST INFRASTRUCTURE ONLY (see the package docstring): imported by ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg, never by the
GPU library.

What is computed (paper passages in brackets):

* An averaged visibility is the boxcar mean of the point-source visibility over
  its time x frequency bin [section 2.3, averaging integral over the sampling
  bin].  Read discretely: the mean over the bin's high-resolution samples.
* Relative to the bin centre it factors as the bin-centre phase times a
  distortion factor [section 3.1, the identity that the sampled distortion is
  the bin-centre phase times the true distortion].  For source direction
  (l0, m0), n0 = sqrt(1 - l0^2 - m0^2), sample s of bin k at uvw u_s (in
  wavelengths) and bin centre u_k:

      phi_s = (u_s - u_k) l0 + (v_s - v_k) m0 + (w_s - w_k)(n0 - 1)
      D_k   = (1/n_k) sum_s exp(-2 pi i phi_s)

  The minus sign follows the paper's forward transform [section 2.1, the
  2-D Fourier relation between sky and visibility].
* Windowed averaging [section 2.3, the boxcar replaced by a baseline-dependent
  window]: with separable sample weights x_s = win_t[b][t] win_c[b][c],
  D_k = sum_s x_s exp(-2 pi i phi_s) / sum_s x_s (0 for a window summing to 0).
* The distorted PSF is the weighted sum over averaged visibilities of their
  inverse transforms [section 2.3, distorted-PSF equation], indexed by the
  offset from the source [section 2.2, direction-dependent convolution].
  With pixel offsets x_i = l_i - l0, y_j = m_j - m0 and the w-term
  linearised about the source (u' = u - w l0/n0, v' = v - w m0/n0), summing
  both conjugate halves of every baseline:

      P_ij = sum_k W_k [D_k exp(2 pi i (u'_k x_i + v'_k y_j)) + c.c.]

* Errors are reported on peak-normalised PSFs [section 4, error in dB of
  normalised PSFs].

Readings taken where the paper is silent (each also listed in the design
notes): the discrete mean over samples rather than the continuous integral;
bin centre = Earth-rotation uvw at the mean sample time and the mean channel
frequency (an input, ``uvw_c_m``); both conjugate halves with equal weight;
the linearised w-shift; pixel grids fixed in absolute (l, m).
"""
from __future__ import annotations

import cmath
import dataclasses
import math
import types

import numpy as np

C_LIGHT = 299792458.0            # m / s
TWO_PI = 2.0 * math.pi
OMEGA_EARTH = 7.2921150e-5       # rad / s, sidereal rotation rate


# --------------------------------------------------------------------------
# bins [section 2.3, sampling bin; bins ordered (baseline, time bin, freq bin)]
# --------------------------------------------------------------------------
@dataclasses.dataclass
class BinTable:
    b: np.ndarray      # [K] baseline of each bin
    t0: np.ndarray     # [K] first sample time index
    t1: np.ndarray     # [K] one past the last
    c0: np.ndarray     # [K] first channel
    c1: np.ndarray     # [K] one past the last
    tb: np.ndarray     # [K] row of the bin-centre uvw table

    @property
    def n(self) -> np.ndarray:
        return (self.t1 - self.t0) * (self.c1 - self.c0)


def bin_table(obs) -> BinTable:
    n_t, n_ch = obs.uvw_m.shape[1], len(obs.freq_hz)
    b_l, t0_l, t1_l, c0_l, c1_l, tb_l = [], [], [], [], [], []
    for b in range(obs.uvw_m.shape[0]):
        nt, nc = int(obs.bl_bin[b, 0]), int(obs.bl_bin[b, 1])
        n_tb, n_fb = -(-n_t // nt), -(-n_ch // nc)
        T = np.repeat(np.arange(n_tb), n_fb)
        F = np.tile(np.arange(n_fb), n_tb)
        b_l.append(np.full(n_tb * n_fb, b))
        t0_l.append(T * nt)
        t1_l.append(np.minimum(n_t, (T + 1) * nt))
        c0_l.append(F * nc)
        c1_l.append(np.minimum(n_ch, (F + 1) * nc))
        tb_l.append(int(obs.bl_tboff[b]) + T)
    cat = lambda xs: np.concatenate(xs).astype(np.int64) if xs else np.zeros(0, np.int64)
    tab = BinTable(cat(b_l), cat(t0_l), cat(t1_l), cat(c0_l), cat(c1_l), cat(tb_l))
    assert len(tab.b) == int(obs.bl_koff[-1]), "bin count disagrees with bl_koff"
    return tab


def _bin_freq(obs, tab: BinTable) -> np.ndarray:
    """Mean channel frequency of every bin (the bin's centre frequency).

    Each distinct channel range [c0, c1) is averaged once with np.mean and
    the value is repeated for every bin with that range (baseline by
    baseline: a baseline's frequency bins repeat in every time bin)."""
    out = np.empty(len(tab.c0))
    cache = {}
    n_ch = len(obs.freq_hz)
    for b in range(obs.uvw_m.shape[0]):
        k0, k1 = int(obs.bl_koff[b]), int(obs.bl_koff[b + 1])
        nc = int(obs.bl_bin[b, 1])
        n_fb = -(-n_ch // nc)
        fm = []
        for F in range(n_fb):
            key = (F * nc, min(n_ch, (F + 1) * nc))
            if key not in cache:
                cache[key] = np.mean(obs.freq_hz[key[0]:key[1]])
            fm.append(cache[key])
        out[k0:k1] = np.tile(np.array(fm), (k1 - k0) // n_fb)
    return out


def bin_centres_lambda(obs, tab: BinTable = None) -> np.ndarray:
    """u_k = uvw at the bin centre, in wavelengths, [K, 3] [section 2.1: u = u(t) nu / c]."""
    tab = bin_table(obs) if tab is None else tab
    nu = _bin_freq(obs, tab)
    return obs.uvw_c_m[tab.tb] * (nu / C_LIGHT)[:, None]


def _lmn(l0: float, m0: float):
    n0 = math.sqrt(1.0 - l0 * l0 - m0 * m0)
    return n0, np.array([l0, m0, n0 - 1.0])


# --------------------------------------------------------------------------
# decorrelation factor
# --------------------------------------------------------------------------
def _per_baseline_phases(obs, tab, uk, b, L):
    """phi for every sample of baseline b and the bin index of each sample."""
    n_t, n_ch = obs.uvw_m.shape[1], len(obs.freq_hz)
    nt, nc = int(obs.bl_bin[b, 0]), int(obs.bl_bin[b, 1])
    n_fb = -(-n_ch // nc)
    k0 = int(obs.bl_koff[b])
    kidx = k0 + (np.arange(n_t)[:, None] // nt) * n_fb + (np.arange(n_ch)[None, :] // nc)
    us = obs.uvw_m[b][:, None, :] * (obs.freq_hz / C_LIGHT)[None, :, None]   # [n_t, n_ch, 3]
    du = us - uk[kidx]                                                           # relative to bin centre
    return du @ L, du, kidx


def _windowed(obs) -> bool:
    return getattr(obs, "win_t", None) is not None or getattr(obs, "win_c", None) is not None


def sample_window(obs, b: int) -> np.ndarray:
    """Window weight of every sample of baseline b, [n_t, n_ch]: the product
    of the time and channel windows (an axis without one is boxcar, 1)."""
    n_t, n_ch = obs.uvw_m.shape[1], len(obs.freq_hz)
    wt = np.ones(n_t) if obs.win_t is None else np.asarray(obs.win_t[b], np.float64)
    wc = np.ones(n_ch) if obs.win_c is None else np.asarray(obs.win_c[b], np.float64)
    return wt[:, None] * wc[None, :]


def _normalise(acc: np.ndarray, wsum: np.ndarray) -> np.ndarray:
    """acc / wsum per bin, 0 where a bin's window sums to 0."""
    out = np.zeros_like(acc)
    nz = wsum != 0.0
    out[..., nz] = acc[..., nz] / wsum[nz]
    return out


def _bin_sum(kidx: np.ndarray, vals: np.ndarray, k0: int, k1: int) -> np.ndarray:
    """Sum of vals per bin over one baseline's bins [k0, k1) (samples in
    their natural order, as np.bincount adds them)."""
    return np.bincount(kidx.ravel() - k0, vals.ravel(), minlength=k1 - k0)


def decorr(obs, l0: float, m0: float, sign: float = -1.0) -> np.ndarray:
    """D_k, complex128 [K]: mean over each bin's samples of exp(sign 2 pi i phi_s).

    sign = -1 is the paper's convention; +1 gives the literal form some
    descriptions use (then every D is conjugated and the PSF is point-mirrored).

    Windowed averaging [section 2.3: the normalised boxcar of the averaging
    integral replaced by a baseline-dependent window X_pqkr]: when the
    observation carries window weights (``win_t`` [n_bl, n_t], ``win_c``
    [n_bl, n_ch]) the mean becomes the window-weighted mean over the bin's
    samples, normalised by the window's sum over the bin, and a bin whose
    window sums to 0 gets D = 0.
    """
    tab = bin_table(obs)
    uk = bin_centres_lambda(obs, tab)
    _, L = _lmn(l0, m0)
    K = len(tab.b)
    re = np.zeros(K)
    im = np.zeros(K)
    if _windowed(obs):
        wsum = np.zeros(K)
        for b in range(obs.uvw_m.shape[0]):
            k0, k1 = int(obs.bl_koff[b]), int(obs.bl_koff[b + 1])
            phi, _, kidx = _per_baseline_phases(obs, tab, uk, b, L)
            x = sample_window(obs, b)
            e = x * np.exp(sign * 1j * TWO_PI * phi)
            re[k0:k1] += _bin_sum(kidx, e.real, k0, k1)
            im[k0:k1] += _bin_sum(kidx, e.imag, k0, k1)
            wsum[k0:k1] += _bin_sum(kidx, x, k0, k1)
        return _normalise(re + 1j * im, wsum)
    for b in range(obs.uvw_m.shape[0]):
        k0, k1 = int(obs.bl_koff[b]), int(obs.bl_koff[b + 1])
        phi, _, kidx = _per_baseline_phases(obs, tab, uk, b, L)
        e = np.exp(sign * 1j * TWO_PI * phi)
        re[k0:k1] += _bin_sum(kidx, e.real, k0, k1)
        im[k0:k1] += _bin_sum(kidx, e.imag, k0, k1)
    return (re + 1j * im) / tab.n


def _step(a: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """Per-sample step of a sampled quantity over samples [lo, hi): the mean
    step between the bin's first and last sample, or, for a one-sample bin,
    the step to its neighbour (zero when the axis has one sample)."""
    n_all = a.shape[0]
    if hi - lo > 1:
        return (a[hi - 1] - a[lo]) / (hi - lo - 1)
    if n_all == 1:
        return np.zeros_like(a[lo])
    return a[lo + 1] - a[lo] if lo + 1 < n_all else a[lo] - a[lo - 1]


def decorr_sinc(obs, l0: float, m0: float) -> np.ndarray:
    """Method 1, the uv-plane approximation [section 3.1]: the distortion of
    bin k replaced by the product of two sincs, sinc(dPsi/2) sinc(dPhi/2),
    where dPsi is the phase change 2 pi du.l0 across the bin's time interval
    at its centre frequency and dPhi the change across its frequency
    interval at its centre time (l0 = (l0, m0): the method is 2-D, w is
    dropped).  sinc(x) = sin(x)/x.  Real, float64 [K].

    Reading (the paper defines the interval by its start and end, not by
    samples): a bin of n samples spaced by s covers n s, so the change across
    it is n times the per-sample step of the track (in time) or of the
    channel frequency (in frequency), the step taken from the bin's own first
    and last samples (from its neighbour for a one-sample bin).
    """
    if _windowed(obs):
        raise ValueError("Method 1 is the closed form of the boxcar average; the observation has windows")
    tab = bin_table(obs)
    nu = _bin_freq(obs, tab)
    L2 = np.array([l0, m0])
    out = np.empty(len(tab.b))
    for k in range(len(tab.b)):
        b = int(tab.b[k])
        t0, t1, c0, c1 = int(tab.t0[k]), int(tab.t1[k]), int(tab.c0[k]), int(tab.c1[k])
        du_time = (t1 - t0) * _step(obs.uvw_m[b], t0, t1)[:2] * (nu[k] / C_LIGHT)       # wavelengths
        dnu = (c1 - c0) * _step(obs.freq_hz, c0, c1)
        du_freq = obs.uvw_c_m[int(tab.tb[k])][:2] * (dnu / C_LIGHT)                     # wavelengths
        x_t = math.pi * float(du_time @ L2)
        x_f = math.pi * float(du_freq @ L2)
        out[k] = np.sinc(x_t / math.pi) * np.sinc(x_f / math.pi)
    return out


def decorr_with_grad(obs, l0: float, m0: float):
    """D_k and its derivatives with respect to l0 and m0.

    d phi/d l0 = du - dw l0/n0 and d phi/d m0 = dv - dw m0/n0, because
    d n0/d l0 = -l0/n0.
    """
    tab = bin_table(obs)
    uk = bin_centres_lambda(obs, tab)
    n0, L = _lmn(l0, m0)
    K = len(tab.b)
    acc = np.zeros((3, K), complex)
    win = _windowed(obs)
    wsum = np.zeros(K)
    for b in range(obs.uvw_m.shape[0]):
        k0, k1 = int(obs.bl_koff[b]), int(obs.bl_koff[b + 1])
        phi, du, kidx = _per_baseline_phases(obs, tab, uk, b, L)
        e = np.exp(-1j * TWO_PI * phi)
        if win:
            x = sample_window(obs, b)
            e = x * e
            wsum[k0:k1] += _bin_sum(kidx, x, k0, k1)
        dphi_l = du[..., 0] - du[..., 2] * l0 / n0
        dphi_m = du[..., 1] - du[..., 2] * m0 / n0
        for r, val in enumerate((e, -1j * TWO_PI * dphi_l * e, -1j * TWO_PI * dphi_m * e)):
            acc[r, k0:k1] += _bin_sum(kidx, val.real, k0, k1) + 1j * _bin_sum(kidx, val.imag, k0, k1)
    if win:
        acc = _normalise(acc, wsum)
    else:
        acc /= tab.n[None, :]
    return acc[0], acc[1], acc[2]


def decorr_brute(obs, l0: float, m0: float, negate: bool = False) -> np.ndarray:
    """D_k by explicit loops over every sample (tiny inputs only).

    ``negate`` evaluates the conjugate baseline qp, whose uvw (samples and
    bin centre) are the negatives of pq's.
    """
    s = -1.0 if negate else 1.0
    n0 = math.sqrt(1.0 - l0 * l0 - m0 * m0)
    tab = bin_table(obs)
    out = np.zeros(len(tab.b), complex)
    wt = getattr(obs, "win_t", None)
    wc = getattr(obs, "win_c", None)
    for k in range(len(tab.b)):
        b, tbrow = int(tab.b[k]), int(tab.tb[k])
        chans = range(int(tab.c0[k]), int(tab.c1[k]))
        nu_c = sum(float(obs.freq_hz[c]) for c in chans) / len(chans)
        uc = [s * float(obs.uvw_c_m[tbrow, a]) * nu_c / C_LIGHT for a in range(3)]
        acc = 0j
        norm = 0.0
        for t in range(int(tab.t0[k]), int(tab.t1[k])):
            for c in chans:
                x = (1.0 if wt is None else float(wt[b, t])) * (1.0 if wc is None else float(wc[b, c]))
                us = [s * float(obs.uvw_m[b, t, a]) * float(obs.freq_hz[c]) / C_LIGHT for a in range(3)]
                phi = (us[0] - uc[0]) * l0 + (us[1] - uc[1]) * m0 + (us[2] - uc[2]) * (n0 - 1.0)
                acc += x * cmath.exp(-2j * math.pi * phi)
                norm += x
        out[k] = acc / norm if norm != 0.0 else 0.0
    return out


# --------------------------------------------------------------------------
# PSF patch
# --------------------------------------------------------------------------
def wshift(uk: np.ndarray, l0: float, m0: float):
    """Linearised w-term: u' = u - w l0/n0, v' = v - w m0/n0."""
    n0 = math.sqrt(1.0 - l0 * l0 - m0 * m0)
    return uk[:, 0] - uk[:, 2] * l0 / n0, uk[:, 1] - uk[:, 2] * m0 / n0


def pixel_offsets(src):
    """x_i = l_i - l0 and y_j = m_j - m0 on the fixed absolute grid."""
    li = src.l_first + np.arange(src.nl) * src.dl
    mj = src.m_first + np.arange(src.nm) * src.dm
    return li - src.l0, mj - src.m0


def patch_factored(obs, src, D: np.ndarray = None, block: int = 8192, sign: float = 1.0) -> np.ndarray:
    """P [nl, nm] float64 = 2 Re sum_k W_k D_k a_ki b_kj.

    The per-term exponential exp(2 pi i (u' x + v' y)) is written as the
    product a_ki b_kj, an exact algebraic regrouping; the sum over k is taken
    block by block only to bound memory.  ``sign`` = -1 flips the sign of the
    imaging exponent (used to check the mirror identity).
    """
    if D is None:
        D = decorr(obs, src.l0, src.m0)
    uk = bin_centres_lambda(obs)
    up, vp = wshift(uk, src.l0, src.m0)
    x, y = pixel_offsets(src)
    c = obs.W.astype(np.float64) * D
    acc = np.zeros((src.nl, src.nm), complex)
    for k0 in range(0, len(c), block):
        sl = slice(k0, k0 + block)
        Ea = np.exp(sign * 1j * TWO_PI * (up[sl, None] * x[None, :]))
        Eb = np.exp(sign * 1j * TWO_PI * (vp[sl, None] * y[None, :]))
        acc += (c[sl, None] * Ea).T @ Eb
    return 2.0 * acc.real


def patch_brute(obs, src) -> np.ndarray:
    """Complex P by brute force: every bin, both baselines pq and qp, every pixel.

    The qp half negates the uvw of samples and bin centre and evaluates its
    own D from those samples; nothing relies on the two halves being
    conjugate.  Returns the complex sum so that callers can check that it is
    real.  Tiny inputs only.
    """
    tab = bin_table(obs)
    n0 = math.sqrt(1.0 - src.l0 ** 2 - src.m0 ** 2)
    li = src.l_first + np.arange(src.nl) * src.dl
    mj = src.m_first + np.arange(src.nm) * src.dm
    X, Y = np.meshgrid(li - src.l0, mj - src.m0, indexing="ij")
    out = np.zeros((src.nl, src.nm), complex)
    for negate in (False, True):
        s = -1.0 if negate else 1.0
        D = decorr_brute(obs, src.l0, src.m0, negate=negate)
        for k in range(len(tab.b)):
            chans = range(int(tab.c0[k]), int(tab.c1[k]))
            nu_c = sum(float(obs.freq_hz[c]) for c in chans) / len(chans)
            u, v, w = (s * float(obs.uvw_c_m[int(tab.tb[k]), a]) * nu_c / C_LIGHT for a in range(3))
            up, vp = u - w * src.l0 / n0, v - w * src.m0 / n0
            out += float(obs.W[k]) * D[k] * np.exp(2j * math.pi * (up * X + vp * Y))
    return out


def patch_pixels(obs, src, ii, jj, D: np.ndarray = None, block: int = 1 << 20) -> np.ndarray:
    """P at the listed pixels only, float64 [len(ii)]."""
    if D is None:
        D = decorr(obs, src.l0, src.m0)
    uk = bin_centres_lambda(obs)
    up, vp = wshift(uk, src.l0, src.m0)
    x, y = pixel_offsets(src)
    c = obs.W.astype(np.float64) * D
    out = np.zeros(len(ii))
    for n, (i, j) in enumerate(zip(ii, jj)):
        acc = 0j
        for k0 in range(0, len(c), block):
            sl = slice(k0, k0 + block)
            acc += np.sum(c[sl] * np.exp(1j * TWO_PI * (up[sl] * x[i] + vp[sl] * y[j])))
        out[n] = 2.0 * acc.real
    return out


def _fullw_offsets(src):
    """x_i, y_j and n(l_i, m_j) - n0 on the patch grid (FP64)."""
    n0 = math.sqrt(1.0 - src.l0 ** 2 - src.m0 ** 2)
    x, y = pixel_offsets(src)
    X, Y = np.meshgrid(x, y, indexing="ij")
    return X, Y, np.sqrt(1.0 - (src.l0 + X) ** 2 - (src.m0 + Y) ** 2) - n0


def patch_fullw(obs, src, D: np.ndarray = None, block: int = 4096) -> np.ndarray:
    """The patch with the exact w phase instead of its linearisation: the
    imaging phase of a bin-centre visibility at pixel (l, m) is
    u l + v m + w (n(l, m) - 1) [section 2.1, the visibility relation with
    its w-term], so relative to the source
        P_ij = sum_k W_k [D_k exp(2 pi i (u_k x_i + v_k y_j + w_k (n_ij - n0))) + c.c.]
    with n_ij = sqrt(1 - l_i^2 - m_j^2).  Not factorable, so evaluated per
    pixel."""
    if D is None:
        D = decorr(obs, src.l0, src.m0)
    uk = bin_centres_lambda(obs)
    X, Y, N = _fullw_offsets(src)
    c = obs.W.astype(np.float64) * D
    acc = np.zeros(X.shape, complex)
    for k0 in range(0, len(c), block):
        sl = slice(k0, k0 + block)
        ph = (uk[sl, 0, None, None] * X[None] + uk[sl, 1, None, None] * Y[None]
              + uk[sl, 2, None, None] * N[None])
        acc += np.tensordot(c[sl], np.exp(1j * TWO_PI * ph), axes=(0, 0))
    return 2.0 * acc.real


def patch_fullw_pixels(obs, src, ii, jj, D: np.ndarray = None, block: int = 1 << 20) -> np.ndarray:
    """``patch_fullw`` at the listed pixels only, float64 [len(ii)]."""
    if D is None:
        D = decorr(obs, src.l0, src.m0)
    uk = bin_centres_lambda(obs)
    X, Y, N = _fullw_offsets(src)
    c = obs.W.astype(np.float64) * D
    out = np.zeros(len(ii))
    for n, (i, j) in enumerate(zip(ii, jj)):
        acc = 0j
        for k0 in range(0, len(c), block):
            sl = slice(k0, k0 + block)
            acc += np.sum(c[sl] * np.exp(1j * TWO_PI * (uk[sl, 0] * X[i, j] + uk[sl, 1] * Y[i, j]
                                                           + uk[sl, 2] * N[i, j])))
        out[n] = 2.0 * acc.real
    return out


# --------------------------------------------------------------------------
# Method 2, the image-plane approximation [section 3.2]
# --------------------------------------------------------------------------
def method2_grid(N: int, cell: float):
    """The centred N x N grid of Method 2 (N even): pixel i at offset
    (i - N/2) cell, and its discrete uv plane: cell a at (a - N/2) du with
    du = 1 / (N cell) [Algorithm 1, the uv cell size from the image extent]."""
    off = (np.arange(N) - N // 2).astype(np.float64)
    return off * cell, off / (N * cell)


def method2_dhat(u0, v0, l0: float, m0: float, dt: float, dnu: float, nu: float):
    """The pixelised decorrelation of Method 2 [section 3.2, the fringe-rate
    model and Algorithm 1] at uv cells (u0, v0) in wavelengths, for a source
    at (l0, m0), bins of dt seconds and dnu Hz at frequency nu:
    a circular track of radius |u0| turning at omega_E has fringe rate
    (du/dt, dv/dt) = omega_E (-v0, u0) (theta the polar angle of (u0, v0),
    as in the track equations), so
        dPsi = 2 pi (du/dt l0 + dv/dt m0) dt,
        dPhi = 2 pi (dnu/nu) |l0| |u0|,
        D^   = sinc(dPsi/2) sinc(dPhi/2),   sinc(x) = sin(x)/x.
    Readings (the algorithm's listing is garbled): uv in wavelengths with no
    further nu/c factor; the direction is the source's (l0, m0); cells step
    by du, not (N-1)/N du."""
    u0 = np.asarray(u0, np.float64)
    v0 = np.asarray(v0, np.float64)
    dpsi = TWO_PI * OMEGA_EARTH * (-v0 * l0 + u0 * m0) * dt
    dphi = TWO_PI * (dnu / nu) * math.hypot(l0, m0) * np.hypot(u0, v0)
    return np.sinc(dpsi / (2.0 * math.pi)) * np.sinc(dphi / (2.0 * math.pi))


def method2_effective_psf(obs, N: int, cell: float) -> np.ndarray:
    """The effective PSF [section 2.2: the PSF at the phase centre, no
    decorrelation] on the centred N x N grid: D = 1, l0 = m0 = 0."""
    x, _ = method2_grid(N, cell)
    grid = types.SimpleNamespace(l0=0.0, m0=0.0, l_first=float(x[0]), m_first=float(x[0]), dl=cell, dm=cell,
                                 nl=N, nm=N)
    return patch_factored(obs, grid, np.ones(int(obs.bl_koff[-1]), complex))


def method2_patch(P_eff: np.ndarray, cell: float, l0: float, m0: float, dt: float, dnu: float,
                  nu: float) -> np.ndarray:
    """Method 2 [section 3.2, the FFT form of the image-plane convolution]:
    the spectrum of the effective PSF on the centred grid times the
    pixelised D^, transformed back; real part, on the same centred grid of
    offsets from the source.  The transforms are the periodic DFT on the
    N x N grid: the edge row and column (offset -N/2) and the Nyquist cells
    (frequency -N/2) are taken as the DFT has them, without symmetrising."""
    N = P_eff.shape[0]
    _, uu = method2_grid(N, cell)
    U, V = np.meshgrid(uu, uu, indexing="ij")
    S = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(P_eff)))
    out = np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(S * method2_dhat(U, V, l0, m0, dt, dnu, nu))))
    return out.real


def patch_normalised(obs, src, D: np.ndarray = None) -> np.ndarray:
    """The normalised PSF [section 4, errors of PSFs normalised at the
    source; Algorithm 2, the properly normalised PSF]: P / P(source), where
    P(source) = 2 Re sum_k W_k D_k is the patch at zero offset (every phase
    factor is 1 there), whether or not the grid holds that pixel."""
    if D is None:
        D = decorr(obs, src.l0, src.m0)
    peak = 2.0 * float(np.sum(obs.W.astype(np.float64) * D.real))
    return patch_factored(obs, src, D) / peak


def peak_normalised_error(P: np.ndarray, ref: np.ndarray):
    """(max |P - ref|, rms(P - ref)) divided by max |ref| [section 4, normalised PSFs]."""
    P = np.asarray(P, np.float64)
    ref = np.asarray(ref, np.float64)
    peak = np.max(np.abs(ref))
    d = P - ref
    return float(np.max(np.abs(d)) / peak), float(np.sqrt(np.mean(d * d)) / peak)


# --------------------------------------------------------------------------
# differentiation of a patch-fitting loss
# --------------------------------------------------------------------------
def _patch_and_derivs(obs, src, block: int = 8192):
    """P and dP/dl0, dP/dm0 on the fixed grid, by differentiating the definition.

    With c_k = W_k D_k, a = exp(2 pi i u' x), b = exp(2 pi i v' y):
      dP/dl0 = 2 Re sum_k [W_k dD_k/dl0 a b
                + c_k 2 pi i (du'/dl0 x_i - u'_k + dv'/dl0 y_j) a b]
    (x_i = l_i - l0 moves with l0), and likewise for m0.
    """
    l0, m0 = src.l0, src.m0
    n0 = math.sqrt(1.0 - l0 * l0 - m0 * m0)
    D, dDl, dDm = decorr_with_grad(obs, l0, m0)
    uk = bin_centres_lambda(obs)
    up, vp = wshift(uk, l0, m0)
    w = uk[:, 2]
    dup_dl = -w * (1.0 - m0 * m0) / n0 ** 3
    dup_dm = -w * l0 * m0 / n0 ** 3
    dvp_dl = dup_dm
    dvp_dm = -w * (1.0 - l0 * l0) / n0 ** 3
    x, y = pixel_offsets(src)
    W = obs.W.astype(np.float64)
    c = W * D
    P = np.zeros((src.nl, src.nm), complex)
    Gl = np.zeros_like(P)
    Gm = np.zeros_like(P)
    for k0 in range(0, len(c), block):
        sl = slice(k0, k0 + block)
        Ea = np.exp(1j * TWO_PI * (up[sl, None] * x[None, :]))
        Eb = np.exp(1j * TWO_PI * (vp[sl, None] * y[None, :]))
        cs = c[sl, None]
        P += (cs * Ea).T @ Eb
        # l0: dD term, du'/dl0 x term, -u' term (from x = l - l0), dv'/dl0 y term
        Gl += ((W[sl, None] * dDl[sl, None]) * Ea).T @ Eb
        Gl += 1j * TWO_PI * ((cs * dup_dl[sl, None] * x[None, :] - cs * up[sl, None]) * Ea).T @ Eb
        Gl += 1j * TWO_PI * (cs * dvp_dl[sl, None] * Ea).T @ (y[None, :] * Eb)
        # m0: dD term, du'/dm0 x term, dv'/dm0 y term, -v' term (from y = m - m0)
        Gm += ((W[sl, None] * dDm[sl, None]) * Ea).T @ Eb
        Gm += 1j * TWO_PI * (cs * dup_dm[sl, None] * x[None, :] * Ea).T @ Eb
        Gm += 1j * TWO_PI * (cs * Ea).T @ ((dvp_dm[sl, None] * y[None, :] - vp[sl, None]) * Eb)
    return 2.0 * P.real, 2.0 * Gl.real, 2.0 * Gm.real


def loss_value(obs, srcs, fluxes, targets) -> float:
    """L = sum_s || f_s P_s(l0_s, m0_s) - T_s ||^2 (the fitting loss of the
    differentiation workload)."""
    tot = 0.0
    for s, f, T in zip(srcs, fluxes, targets):
        r = f * patch_factored(obs, s) - T
        tot += float(np.sum(r * r))
    return tot


def loss_grad_analytic(obs, srcs, fluxes, targets):
    """(L, dL/d(l0, m0) [n_src, 2], dL/dflux [n_src]) from the derivative patches."""
    g_lm = np.zeros((len(srcs), 2))
    g_f = np.zeros(len(srcs))
    L = 0.0
    for n, (s, f, T) in enumerate(zip(srcs, fluxes, targets)):
        P, dl, dm = _patch_and_derivs(obs, s)
        r = f * P - T
        L += float(np.sum(r * r))
        G = 2.0 * f * r
        g_lm[n] = (np.sum(G * dl), np.sum(G * dm))
        g_f[n] = 2.0 * np.sum(r * P)
    return L, g_lm, g_f


def loss_grad_fd(obs, srcs, fluxes, targets, h: float = 1e-3 * math.pi / (180 * 3600)):
    """Central finite differences of ``loss_value`` in l0 and m0 of every
    source (grid fixed), step h (default 1e-3 arcsec)."""
    g = np.zeros((len(srcs), 2))
    for n, (s, f, T) in enumerate(zip(srcs, fluxes, targets)):
        for a in range(2):
            vals = []
            for sgn in (+1.0, -1.0):
                l0 = s.l0 + (sgn * h if a == 0 else 0.0)
                m0 = s.m0 + (sgn * h if a == 1 else 0.0)
                r = f * patch_factored(obs, s.with_direction(l0, m0)) - T
                vals.append(float(np.sum(r * r)))
            g[n, a] = (vals[0] - vals[1]) / (2.0 * h)
    return g


# --------------------------------------------------------------------------
# deconvolution with position-dependent PSFs [Algorithm 2, Hogbom CLEAN]
# --------------------------------------------------------------------------
def hogbom_clean_method2(P_eff: np.ndarray, grid, dirty: np.ndarray, gain: float, n_iter: int, dt: float,
                         dnu: float, nu: float, threshold: float = 0.0):
    """Hogbom CLEAN [Algorithm 2] with the Method-2 PSF at every peak
    [section 3.2]: the PSF of the peak pixel's direction is
    ``method2_patch(P_eff, ...)`` on the centred N x N grid of offsets (the
    image's cell, square), laid with its centre on the peak pixel; image
    pixels beyond its extent are not changed.  Peak rule, normalisation at
    the peak and update as in ``hogbom_clean``.  Returns (residual,
    [(i, j, amp)])."""
    N = P_eff.shape[0]
    h = N // 2
    res = np.array(dirty, dtype=np.float64)
    nl, nm = res.shape
    comps = []
    for _ in range(n_iter):
        flat = int(np.argmax(np.abs(res)))
        i, j = divmod(flat, nm)
        peak = res[i, j]
        if abs(peak) < threshold:
            break
        Q = method2_patch(P_eff, grid.dl, grid.l_first + i * grid.dl, grid.m_first + j * grid.dm, dt, dnu, nu)
        a0, a1 = max(0, i - h), min(nl, i - h + N)
        b0, b1 = max(0, j - h), min(nm, j - h + N)
        placed = np.zeros_like(res)
        placed[a0:a1, b0:b1] = Q[a0 - i + h:a1 - i + h, b0 - j + h:b1 - j + h]
        res = res - gain * peak * placed / Q[h, h]
        comps.append((i, j, gain * peak))
    return res, comps


def hogbom_clean(obs, grid, dirty: np.ndarray, gain: float, n_iter: int, threshold: float = 0.0,
                 D_of=None):
    """Hogbom CLEAN in which every minor cycle computes the distorted PSF at
    the current peak [Algorithm 2]: find the peak pixel of |residual|, form
    P_d at that direction on the image grid (``grid``: l_first, m_first, dl,
    dm, nl, nm), subtract gain * peak * P_d / P_d(peak), record the component
    gain * peak; stop after n_iter cycles or when |peak| < threshold.  (The
    model update accumulates: the listing assigns it.)  The peak is the first
    maximum in row-major order.  ``D_of(l0, m0)`` may supply the decorrelation
    factors (default: the exact ones).  Returns (residual, [(i, j, amp)])."""
    res = np.array(dirty, dtype=np.float64)
    comps = []
    for _ in range(n_iter):
        flat = int(np.argmax(np.abs(res)))
        i, j = divmod(flat, res.shape[1])
        peak = res[i, j]
        if abs(peak) < threshold:
            break
        l0 = grid.l_first + i * grid.dl
        m0 = grid.m_first + j * grid.dm
        src = grid.with_direction(l0, m0)
        P = patch_factored(obs, src, None if D_of is None else D_of(l0, m0))
        res = res - gain * peak * P / P[i, j]
        comps.append((i, j, gain * peak))
    return res, comps
