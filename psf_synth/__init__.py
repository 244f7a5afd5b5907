"""Seeded synthetic observations shaped like the paper's MeerKAT simulation.

This module produces *input data only*: antenna layouts, Earth-rotation uvw
tracks in metres, channel frequencies, the table of averaging bins, the
weights and the source/patch lists.  It evaluates no decorrelation factor and
no PSF.  Both the FP64 CPU reference (``oracle/``) and the GPU library take
the arrays built here as their inputs, and neither shares any arithmetic of
the method with this module.

Conventions (all fixed here, because the paper does not state them):

* Sample times are integration midpoints symmetric about transit,
  ``t_j = -T/2 + (j + 1/2) dt``; hour angle ``H = omega_E t``.
* Channel centres are ``nu_c = nu_lo + (c + 1/2) dnu``.
* uvw follow the textbook Earth-rotation relation (Thompson, Moran & Swenson,
  the reference the paper cites in its section 2.1): ENU baseline -> equatorial
  (X, Y, Z) at latitude phi, then rotation by hour angle H and declination
  delta.
* A baseline b = (p, q), p < q, has ENU vector pos[q] - pos[p].
* Bins of baseline b hold ``nt_b`` consecutive samples in time and ``nc_b``
  consecutive channels; they tile from the first sample, the last bin in
  each direction may be short.  Bins are ordered (baseline, time bin,
  frequency bin), so bin k of baseline b with time bin T and frequency bin F
  is ``k = koff[b] + T * n_fb(b) + F``.
* The bin-centre uvw of time bin T is the Earth-rotation uvw at the mean of
  the bin's sample times (not the mean of the sample uvw); for a one-sample
  bin it is that sample's row, copied bit for bit.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

OMEGA_EARTH = 7.2921150e-5          # rad / s, sidereal rotation rate
ARCSEC = math.pi / (180.0 * 3600.0)  # radians per arcsecond
DEG = math.pi / 180.0

LATITUDE = -30.7 * DEG               # MeerKAT-like site latitude
DECLINATION = -30.0 * DEG            # phase-centre declination


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Observation:
    """One synthetic observation: every array the library's ABI takes."""
    ant_enu: np.ndarray        # [n_ant, 3] metres (E, N, U)
    bl_ant: np.ndarray         # [n_bl, 2] int32 antenna pair (p, q), p < q
    times_s: np.ndarray        # [n_t] sample times (s), midpoints
    uvw_m: np.ndarray          # [n_bl, n_t, 3] float64 metres
    freq_hz: np.ndarray        # [n_ch] float64 channel centres
    bl_bin: np.ndarray         # [n_bl, 2] int32 {nt_b, nc_b}
    bl_koff: np.ndarray        # [n_bl + 1] int64 first bin of each baseline
    bl_tboff: np.ndarray       # [n_bl + 1] int64 first time-bin row of each baseline
    uvw_c_m: np.ndarray        # [n_tb, 3] float64 bin-centre uvw (metres)
    W: np.ndarray              # [K] float32 weights
    name: str = "custom"
    win_t: Optional[np.ndarray] = None   # [n_bl, n_t] float32 time-window weights, None = boxcar
    win_c: Optional[np.ndarray] = None   # [n_bl, n_ch] float32 channel-window weights, None = boxcar

    @property
    def n_bl(self) -> int:
        return int(self.uvw_m.shape[0])

    @property
    def n_t(self) -> int:
        return int(self.uvw_m.shape[1])

    @property
    def n_ch(self) -> int:
        return int(self.freq_hz.shape[0])

    @property
    def K(self) -> int:
        return int(self.bl_koff[-1])

    @property
    def n_tb(self) -> int:
        return int(self.bl_tboff[-1])

    @property
    def n_samples(self) -> int:
        return self.n_bl * self.n_t * self.n_ch


@dataclasses.dataclass
class Source:
    """A source direction and the absolute pixel grid of its PSF patch.

    Pixel (i, j) sits at l = l_first + i*dl, m = m_first + j*dm.  The output
    patch is row-major [nl][nm] with i along l (east) and j along m (north).
    """
    l0: float
    m0: float
    l_first: float
    m_first: float
    dl: float
    dm: float
    nl: int
    nm: int
    flux: float = 1.0

    @staticmethod
    def centred(l0: float, m0: float, n: int, cell_rad: float,
                nm: Optional[int] = None, flux: float = 1.0) -> "Source":
        nm = n if nm is None else nm
        return Source(l0=l0, m0=m0,
                      l_first=l0 - 0.5 * (n - 1) * cell_rad,
                      m_first=m0 - 0.5 * (nm - 1) * cell_rad,
                      dl=cell_rad, dm=cell_rad, nl=n, nm=nm, flux=flux)

    def with_direction(self, l0: float, m0: float) -> "Source":
        """Same absolute grid, different source direction."""
        return dataclasses.replace(self, l0=l0, m0=m0)


# --------------------------------------------------------------------------
# random streams
# --------------------------------------------------------------------------
def rng(config: int, stream: int, seed: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(config), int(stream), int(seed)]))


STREAM_LAYOUT, STREAM_WEIGHTS, STREAM_SOURCES, STREAM_PERTURB, STREAM_SIZES = range(5)


# --------------------------------------------------------------------------
# layouts
# --------------------------------------------------------------------------
def layout_disc(n_ant: int, radius_m: float, g: np.random.Generator) -> np.ndarray:
    """Antennas uniform in area inside a disc, Up = 0."""
    r = radius_m * np.sqrt(g.random(n_ant))
    th = 2.0 * math.pi * g.random(n_ant)
    return np.stack([r * np.cos(th), r * np.sin(th), np.zeros(n_ant)], axis=1)


def layout_meerkat_like(g: np.random.Generator, n_core: int = 48, n_outer: int = 16,
                        core_sigma_m: float = 300.0, r_in_m: float = 1000.0,
                        r_out_m: float = 4000.0) -> np.ndarray:
    """Gaussian core (isotropic, sigma per axis) plus an area-uniform annulus."""
    core = g.normal(0.0, core_sigma_m, size=(n_core, 2))
    r = np.sqrt(g.uniform(r_in_m ** 2, r_out_m ** 2, size=n_outer))
    th = 2.0 * math.pi * g.random(n_outer)
    outer = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    en = np.concatenate([core, outer], axis=0)
    return np.concatenate([en, np.zeros((en.shape[0], 1))], axis=1)


def baselines(ant_enu: np.ndarray):
    n = ant_enu.shape[0]
    p, q = np.triu_indices(n, k=1)
    return np.stack([p, q], axis=1).astype(np.int32), ant_enu[q] - ant_enu[p]


# --------------------------------------------------------------------------
# Earth rotation
# --------------------------------------------------------------------------
def enu_to_xyz(enu: np.ndarray, lat: float) -> np.ndarray:
    e, n, u = enu[..., 0], enu[..., 1], enu[..., 2]
    x = -n * math.sin(lat) + u * math.cos(lat)
    y = e
    z = n * math.cos(lat) + u * math.sin(lat)
    return np.stack([x, y, z], axis=-1)


def uvw_tracks(bl_enu: np.ndarray, hour_angle: np.ndarray, lat: float = LATITUDE,
               dec: float = DECLINATION) -> np.ndarray:
    """uvw in metres, shape [n_bl, n_h, 3], for hour angles in radians."""
    xyz = enu_to_xyz(bl_enu, lat)
    X, Y, Z = xyz[:, 0:1], xyz[:, 1:2], xyz[:, 2:3]
    sh, ch = np.sin(hour_angle)[None, :], np.cos(hour_angle)[None, :]
    sd, cd = math.sin(dec), math.cos(dec)
    u = X * sh + Y * ch
    v = -X * sd * ch + Y * sd * sh + Z * cd
    w = X * cd * ch - Y * cd * sh + Z * sd
    return np.stack([u, v, w], axis=-1)


def sample_times(n_t: int, dt: float) -> np.ndarray:
    return -0.5 * n_t * dt + (np.arange(n_t) + 0.5) * dt


def channel_centres(nu_lo: float, nu_hi: float, n_ch: int) -> np.ndarray:
    dnu = (nu_hi - nu_lo) / n_ch
    return nu_lo + (np.arange(n_ch) + 0.5) * dnu


# --------------------------------------------------------------------------
# bins
# --------------------------------------------------------------------------
def bin_tables(n_t: int, n_ch: int, bl_bin: np.ndarray):
    nt = bl_bin[:, 0].astype(np.int64)
    nc = bl_bin[:, 1].astype(np.int64)
    n_tb = -(-n_t // nt)
    n_fb = -(-n_ch // nc)
    koff = np.zeros(len(nt) + 1, np.int64)
    koff[1:] = np.cumsum(n_tb * n_fb)
    tboff = np.zeros(len(nt) + 1, np.int64)
    tboff[1:] = np.cumsum(n_tb)
    return koff, tboff


def bin_centre_uvw(bl_enu: np.ndarray, times: np.ndarray, uvw_m: np.ndarray,
                   bl_bin: np.ndarray, lat: float, dec: float) -> np.ndarray:
    """Earth-rotation uvw at the mean time of every time bin, [n_tb, 3].

    Baselines sharing a bin length are done together: the mean time of
    each full bin is a row mean of the reshaped time axis (the same sum as
    the mean of the slice), the short last bin is averaged on its own.
    """
    n_t = times.shape[0]
    nts = bl_bin[:, 0].astype(np.int64)
    off = np.zeros(len(nts) + 1, np.int64)
    off[1:] = np.cumsum(-(-n_t // nts))
    out = np.empty((int(off[-1]), 3))
    for nt in np.unique(nts):
        nt = int(nt)
        bls = np.nonzero(nts == nt)[0]
        n_tb, n_full = -(-n_t // nt), n_t // nt
        t_centre = np.empty(n_tb)
        t_centre[:n_full] = np.mean(times[:n_full * nt].reshape(n_full, nt), axis=1)
        if n_tb > n_full:
            t_centre[n_full] = np.mean(times[n_full * nt:])
        uc = uvw_tracks(bl_enu[bls], OMEGA_EARTH * t_centre, lat, dec)    # [n, n_tb, 3]
        single = np.minimum(n_t, (np.arange(n_tb) + 1) * nt) - np.arange(n_tb) * nt == 1
        if single.any():
            # one-sample bins: the centre is the sample itself, bit for bit
            idx = np.nonzero(single)[0]
            uc[:, idx] = uvw_m[bls][:, idx * nt]
        for q, b in enumerate(bls):
            out[off[b]:off[b + 1]] = uc[q]
    return out


def bin_centre_uvw_uniform(bl_enu: np.ndarray, times: np.ndarray, uvw_m: np.ndarray,
                           nt: int, lat: float, dec: float) -> np.ndarray:
    """Vectorised ``bin_centre_uvw`` for the case of one bin length for all baselines."""
    n_t = times.shape[0]
    n_tb = -(-n_t // nt)
    t_centre = np.array([np.mean(times[T * nt:min(n_t, (T + 1) * nt)]) for T in range(n_tb)])
    uc = uvw_tracks(bl_enu, OMEGA_EARTH * t_centre, lat, dec)          # [n_bl, n_tb, 3]
    single = np.array([min(n_t, (T + 1) * nt) - T * nt == 1 for T in range(n_tb)])
    if single.any():
        idx = np.nonzero(single)[0]
        uc[:, idx] = uvw_m[:, idx * nt]
    return uc.reshape(-1, 3)


def make_observation(ant_enu: np.ndarray, n_t: int, dt: float, freq_hz: np.ndarray,
                     bl_bin, weights: Optional[np.ndarray] = None,
                     lat: float = LATITUDE, dec: float = DECLINATION,
                     weight_rng: Optional[np.random.Generator] = None,
                     weight_range=(0.5, 1.5), name: str = "custom") -> Observation:
    bl_ant, bl_enu = baselines(np.asarray(ant_enu, np.float64))
    n_bl = bl_ant.shape[0]
    times = sample_times(n_t, dt)
    uvw_m = uvw_tracks(bl_enu, OMEGA_EARTH * times, lat, dec)
    bl_bin = np.asarray(bl_bin, np.int32)
    if bl_bin.ndim == 1:
        bl_bin = np.tile(bl_bin[None, :], (n_bl, 1)).astype(np.int32)
    koff, tboff = bin_tables(n_t, len(freq_hz), bl_bin)
    if np.all(bl_bin == bl_bin[0:1]):
        uvw_c = bin_centre_uvw_uniform(bl_enu, times, uvw_m, int(bl_bin[0, 0]), lat, dec)
    else:
        uvw_c = bin_centre_uvw(bl_enu, times, uvw_m, bl_bin, lat, dec)
    K = int(koff[-1])
    if weights is None:
        if weight_rng is None:
            W = np.ones(K, np.float32)
        else:
            W = weight_rng.uniform(weight_range[0], weight_range[1], size=K).astype(np.float32)
    else:
        W = np.asarray(weights, np.float32)
        assert W.shape == (K,)
    return Observation(ant_enu=np.asarray(ant_enu, np.float64), bl_ant=bl_ant, times_s=times,
                       uvw_m=np.ascontiguousarray(uvw_m), freq_hz=np.asarray(freq_hz, np.float64),
                       bl_bin=bl_bin, bl_koff=koff, bl_tboff=tboff,
                       uvw_c_m=np.ascontiguousarray(uvw_c), W=W, name=name)


def bda_bins(bl_enu: np.ndarray, max_t: int = 64, max_c: int = 8) -> np.ndarray:
    """Baseline-dependent bin lengths: floor(B_max/|b|) clamped per axis."""
    L = np.linalg.norm(bl_enu, axis=1)
    r = np.floor(L.max() / L).astype(np.int64)
    nt = np.clip(r, 1, max_t)
    nc = np.clip(r, 1, max_c)
    return np.stack([nt, nc], axis=1).astype(np.int32)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------
CONFIG_NAMES = {
    1: "tiny: 7 ants in 1 km, 600 x 1 s, 1 ch at 1.4 GHz, 30-sample bins, 65^2 at 2\"",
    2: "MeerKAT-shaped: 64 ants, 3600 x 2 s, 32 ch 1.3-1.5 GHz, 10x4 bins, 257^2 at 1.5\"",
    3: "differentiation: config-2 data, 16 sources, 129^2 at 1.5\"",
    4: "precision: 64 ants, 1800 x 2 s, 64 ch 0.9-1.7 GHz, 5x2 bins, 64 sources, 257^2",
    5: "batched BDA: 64 ants, 14400 x 1 s, 64 ch 1.3-1.5 GHz, BDA bins, 256 sources",
    6: "the paper's averaging setup: 64 ants, 7200 x 1 s, 120 x 50 kHz ch at 1.4 GHz, 20 s x 2 MHz bins",
}


def observation(config: int, seed: int = 0, bin_samples: Optional[int] = None) -> Observation:
    """The observation of workload ``config`` (1..6).

    ``bin_samples`` overrides the time-bin length of workload 1 (30 by
    default; 20 gives the 630-bin variant).
    """
    g = rng(config if config not in (3, 6) else 2, STREAM_LAYOUT, seed)
    if config == 1:
        ants = layout_disc(7, 1000.0, g)
        nt = 30 if bin_samples is None else int(bin_samples)
        return make_observation(ants, 600, 1.0, np.array([1.4e9]), [nt, 1], name="config1")
    ants = layout_meerkat_like(g)
    wr = rng(config, STREAM_WEIGHTS, seed)
    if config in (2, 3):
        return make_observation(ants, 3600, 2.0, channel_centres(1.3e9, 1.5e9, 32), [10, 4],
                                weight_rng=wr, name=f"config{config}")
    if config == 4:
        return make_observation(ants, 1800, 2.0, channel_centres(0.9e9, 1.7e9, 64), [5, 2],
                                weight_rng=wr, name="config4")
    if config == 5:
        _, bl_enu = baselines(ants)
        return make_observation(ants, 14400, 1.0, channel_centres(1.3e9, 1.5e9, 64),
                                bda_bins(bl_enu), weight_rng=wr, name="config5")
    if config == 6:
        # 2 h at 1 s, 6 MHz of 120 x 50 kHz channels centred on 1.4 GHz,
        # averaged to 20 s x 2 MHz (40 channels), natural weights
        return make_observation(ants, 7200, 1.0, channel_centres(1.397e9, 1.403e9, 120), [20, 40],
                                name="config6")
    raise ValueError(f"unknown workload {config}")


def direction(r_rad: float, pa_rad: float):
    """Direction cosines of a source at angular radius r and position angle pa."""
    s = math.sin(r_rad)
    return s * math.sin(pa_rad), s * math.cos(pa_rad)


def sources(config: int, seed: int = 0) -> List[Source]:
    g = rng(config, STREAM_SOURCES, seed)
    if config == 1:
        return [Source.centred(0.5 * DEG, 0.3 * DEG, 65, 2.0 * ARCSEC)]
    if config == 2:
        l0, m0 = direction(1.0 * DEG, 2.0 * math.pi * g.random())
        return [Source.centred(l0, m0, 257, 1.5 * ARCSEC)]
    if config == 3:
        out = []
        for _ in range(16):
            r = g.uniform(0.2, 2.0) * DEG
            l0, m0 = direction(r, 2.0 * math.pi * g.random())
            flux = 10.0 ** g.uniform(-2.0, 0.0)
            out.append(Source.centred(l0, m0, 129, 1.5 * ARCSEC, flux=flux))
        return out
    if config == 4:
        out = []
        for _ in range(64):
            l0, m0 = direction(g.uniform(0.1, 3.0) * DEG, 2.0 * math.pi * g.random())
            out.append(Source.centred(l0, m0, 257, 1.5 * ARCSEC))
        return out
    if config == 5:
        gs = rng(config, STREAM_SIZES, seed)
        out = []
        for _ in range(256):
            l0, m0 = direction(g.uniform(0.05, 3.0) * DEG, 2.0 * math.pi * g.random())
            n = int(gs.choice([65, 129, 257]))
            out.append(Source.centred(l0, m0, n, 1.5 * ARCSEC))
        return out
    raise ValueError(f"unknown workload {config}")


def perturbed_targets(config: int, srcs: Sequence[Source], seed: int = 0, sigma_arcsec: float = 1.0):
    """Positions for the differentiation targets: each source moved by N(0, sigma) per axis."""
    g = rng(config, STREAM_PERTURB, seed)
    out = []
    for s in srcs:
        dl, dm = g.normal(0.0, sigma_arcsec * ARCSEC, size=2)
        out.append(s.with_direction(s.l0 + dl, s.m0 + dm))
    return out


def first_baselines(obs: Observation, n_bl: int) -> Observation:
    """The same observation restricted to its first ``n_bl`` baselines (a
    bounded sample of a large workload)."""
    B = min(int(n_bl), obs.n_bl)
    k1, tb1 = int(obs.bl_koff[B]), int(obs.bl_tboff[B])
    return Observation(ant_enu=obs.ant_enu, bl_ant=obs.bl_ant[:B], times_s=obs.times_s,
                       uvw_m=obs.uvw_m[:B], freq_hz=obs.freq_hz, bl_bin=obs.bl_bin[:B],
                       bl_koff=obs.bl_koff[:B + 1], bl_tboff=obs.bl_tboff[:B + 1],
                       uvw_c_m=obs.uvw_c_m[:tb1], W=obs.W[:k1], name=f"{obs.name}[:{B}]",
                       win_t=None if obs.win_t is None else obs.win_t[:B],
                       win_c=None if obs.win_c is None else obs.win_c[:B])


def _bin_position(n: int, size: np.ndarray) -> np.ndarray:
    """Centre offset of every sample inside its bin as a fraction of the
    bin's own span, in (-1/2, 1/2): [n_bl, n] for bins of ``size[b]``
    samples tiling from the first sample (the last bin may be short)."""
    idx = np.arange(n)[None, :]
    size = np.asarray(size, np.int64)[:, None]
    first = (idx // size) * size
    span = np.minimum(size, n - first)
    return (idx - first + 0.5) / span - 0.5


def tapered_windows(obs: Observation, strength: float = 1.0, channels: bool = True) -> Observation:
    """A copy of ``obs`` with baseline-dependent, separable averaging windows
    (input data for windowed averaging; the paper leaves the window shape to
    the cited window designs).  Per axis, a sample at centre offset x of its
    bin (a fraction of the bin span) has weight (1 - a) + a cos^2(pi x),
    a = strength |b| / max |b|: close to the boxcar on short baselines, a
    raised cosine on the longest.  ``channels=False`` leaves the channel axis
    boxcar."""
    bl_enu = obs.ant_enu[obs.bl_ant[:, 1]] - obs.ant_enu[obs.bl_ant[:, 0]]
    L = np.linalg.norm(bl_enu, axis=1)
    a = (float(strength) * L / L.max())[:, None]
    xt = _bin_position(obs.n_t, obs.bl_bin[:, 0])
    win_t = ((1.0 - a) + a * np.cos(math.pi * xt) ** 2).astype(np.float32)
    if channels:
        xc = _bin_position(obs.n_ch, obs.bl_bin[:, 1])
        win_c = ((1.0 - a) + a * np.cos(math.pi * xc) ** 2).astype(np.float32)
    else:
        win_c = None
    return dataclasses.replace(obs, win_t=np.ascontiguousarray(win_t),
                               win_c=None if win_c is None else np.ascontiguousarray(win_c),
                               name=f"{obs.name}+win{strength:g}")


# --------------------------------------------------------------------------
# small random observations for property tests and edge cases
# --------------------------------------------------------------------------
def tiny_random(seed: int, n_ant: int = 4, n_t: int = 7, n_ch: int = 3, nt: int = 3, nc: int = 2,
                radius_m: float = 3000.0, dt: float = 8.0, nu_lo: float = 1.3e9,
                nu_hi: float = 1.5e9, bda: bool = False) -> Observation:
    g = rng(100, STREAM_LAYOUT, seed)
    ants = layout_disc(n_ant, radius_m, g)
    ants[:, 2] = g.normal(0.0, 30.0, n_ant)        # give w a non-trivial height term
    freqs = channel_centres(nu_lo, nu_hi, n_ch)
    if bda:
        _, bl_enu = baselines(ants)
        bins = bda_bins(bl_enu, max_t=nt, max_c=nc)
    else:
        bins = [nt, nc]
    return make_observation(ants, n_t, dt, freqs, bins, weight_rng=rng(100, STREAM_WEIGHTS, seed),
                            name=f"tiny{seed}")
