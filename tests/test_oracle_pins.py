"""Pins of the FP64 CPU reference against facts fixed by the paper and by
mathematics (CPU only).  Each test is chosen so that a plausible mistake in
the reference (dropped term, wrong sign, swapped l/m, wrong bin centre,
missing conjugate half, missing w-shift) fails at least one of them."""
import math
import os

import numpy as np
import pytest

import oracle as orc
import psf_synth as ps

HERE = os.path.dirname(os.path.abspath(__file__))
C = 299792458.0


# ---------------------------------------------------------------- helpers
def ramp_observation(n_samples, bin_len, g_m_per_sample, nu=1.4e9, axis=0, n_ch=1,
                     bin_ch=1, dnu=0.0, u0=(1234.5, -321.0, 45.0)):
    """One baseline whose uvw run linearly in time (slope g along ``axis``),
    channels spaced by dnu.  The bin centre is the exact centre of the ramp."""
    j = np.arange(n_samples, dtype=np.float64)
    uvw = np.tile(np.asarray(u0, np.float64), (n_samples, 1))
    uvw[:, axis] += g_m_per_sample * j
    n_tb = -(-n_samples // bin_len)
    centre = np.tile(np.asarray(u0, np.float64), (n_tb, 1))
    for T in range(n_tb):
        jj = j[T * bin_len:min(n_samples, (T + 1) * bin_len)]
        centre[T, axis] += g_m_per_sample * jj.mean()
    freqs = nu + dnu * (np.arange(n_ch) - 0.5 * (n_ch - 1))
    bl_bin = np.array([[bin_len, bin_ch]], np.int32)
    koff, tboff = ps.bin_tables(n_samples, n_ch, bl_bin)
    return ps.Observation(ant_enu=np.zeros((2, 3)), bl_ant=np.array([[0, 1]], np.int32),
                          times_s=j, uvw_m=uvw[None], freq_hz=freqs, bl_bin=bl_bin,
                          bl_koff=koff, bl_tboff=tboff, uvw_c_m=centre,
                          W=np.ones(int(koff[-1]), np.float32))


def dirichlet(n, d):
    if abs(math.sin(math.pi * d)) < 1e-300:
        return 1.0
    return math.sin(n * math.pi * d) / (n * math.sin(math.pi * d))


def load_dirichlet_pins():
    rows = []
    with open(os.path.join(HERE, "golden", "dirichlet_pins.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                n, d, D = line.split()
                rows.append((int(n), float(d), float(D)))
    return rows


@pytest.fixture(scope="module")
def cfg1():
    obs = ps.observation(1)
    src = ps.sources(1)[0]
    return obs, src


@pytest.fixture(scope="module")
def tiny():
    return ps.tiny_random(3, n_ant=4, n_t=7, n_ch=3, nt=3, nc=2)


# ---------------------------------------------------------------- D_k
def test_D_is_one_at_phase_centre(cfg1):
    # Section 4: at l0 = 0 the averaged visibilities carry no decorrelation.
    obs, _ = cfg1
    D = orc.decorr(obs, 0.0, 0.0)
    assert np.array_equal(D, np.ones_like(D))


def test_D_is_one_for_single_sample_bins():
    obs = ps.tiny_random(5, n_t=5, n_ch=3, nt=1, nc=1)
    D = orc.decorr(obs, 0.02, -0.03)
    assert np.array_equal(D, np.ones_like(D))


@pytest.mark.parametrize("n,d,expect", load_dirichlet_pins())
def test_linear_ramp_matches_dirichlet_golden(n, d, expect):
    # A time ramp: per-sample phase step d turns = g nu l0 / c.
    nu, l0 = 1.4e9, 0.01
    g = d * C / (nu * l0)
    obs = ramp_observation(3 * n, n, g, nu=nu, axis=0)
    D = orc.decorr(obs, l0, 0.0)
    assert np.allclose(D.real, expect, atol=1e-12, rtol=0)
    assert np.max(np.abs(D.imag)) < 1e-12


@pytest.mark.parametrize("n", [3, 8, 17])
def test_frequency_ramp_matches_dirichlet(n):
    # Channels spaced dnu at fixed uvw: phase step u dnu m0 / c per channel.
    nu, m0, dnu = 1.4e9, -0.02, 5e6
    obs = ramp_observation(2, 1, 0.0, nu=nu, n_ch=2 * n, bin_ch=n, dnu=dnu, u0=(300.0, 2100.0, 0.0))
    D = orc.decorr(obs, 0.0, m0)
    d = 2100.0 * dnu * m0 / C
    assert np.allclose(D, dirichlet(n, d), atol=1e-12, rtol=0)


@pytest.mark.parametrize("x", [0.4, 1.3, 2.9])
def test_discrete_mean_tends_to_paper_sinc(x):
    # Section 3.1: boxcar average -> sinc(dPsi/2).  The discrete mean over n
    # samples is x/(n sin(x/n)) * sinc(x), x = dPsi/2, i.e. relative gap
    # x^2/(6 n^2) + O(n^-4).
    nu, l0 = 1.4e9, 0.01
    for n in (16, 64, 256):
        d = x / (n * math.pi)
        g = d * C / (nu * l0)
        D = orc.decorr(ramp_observation(n, n, g, nu=nu), l0, 0.0)[0].real
        sinc = math.sin(x) / x
        rel = D / sinc - 1.0
        assert abs(rel - x * x / (6 * n * n)) < 0.02 * x ** 4 / n ** 4 + 1e-12


def test_earth_rotation_D_close_to_paper_sinc():
    # On true Earth-rotation tracks D is not exactly a ramp; the paper's
    # Method-1 closed form sinc(dPsi/2) sinc(dPhi/2) with dPsi over the bin's
    # time span must still agree to ~1e-5 for 20-30 s bins at 1 km.
    obs = ps.observation(1)
    l0, m0 = 0.5 * ps.DEG, 0.3 * ps.DEG
    D = orc.decorr(obs, l0, m0)
    tab = orc.bin_table(obs)
    _, bl_enu = ps.baselines(obs.ant_enu)
    dt = obs.times_s[1] - obs.times_s[0]
    nu = obs.freq_hz[0]
    n0 = math.sqrt(1 - l0 * l0 - m0 * m0)
    ts = obs.times_s[tab.t0] - 0.5 * dt
    te = obs.times_s[tab.t1 - 1] + 0.5 * dt
    us = np.stack([ps.uvw_tracks(bl_enu[b:b + 1], np.array([ps.OMEGA_EARTH * t]))[0, 0] for b, t in zip(tab.b, ts)])
    ue = np.stack([ps.uvw_tracks(bl_enu[b:b + 1], np.array([ps.OMEGA_EARTH * t]))[0, 0] for b, t in zip(tab.b, te)])
    dpsi = 2 * math.pi * ((us - ue) @ np.array([l0, m0, n0 - 1])) * nu / C
    x = dpsi / 2
    sinc = np.sinc(x / math.pi)                  # np.sinc(y) = sin(pi y)/(pi y)
    n = (tab.t1 - tab.t0).astype(np.float64)
    dirich = np.sin(x) / (n * np.sin(x / n))     # discrete mean of the same ramp
    # the discrete mean sits x^2/(6 n^2) above the paper's continuous sinc ...
    assert np.max(np.abs(D.real - sinc)) < 2e-5
    assert np.allclose(D.real / sinc - 1, x * x / (6 * n * n), rtol=0.05, atol=1e-9)
    # ... and equals the Dirichlet form up to the tracks' small curvature
    assert np.max(np.abs(D.real - dirich)) < 1e-8
    assert np.max(np.abs(D.imag)) < 1e-4


def test_decorr_matches_explicit_loops(tiny):
    D = orc.decorr(tiny, 0.031, -0.017)
    Db = orc.decorr_brute(tiny, 0.031, -0.017)
    assert np.max(np.abs(D - Db)) < 1e-12      # FP64 rounding of u ~ 1e4 wavelengths


def test_decorr_sign_convention(tiny):
    D = orc.decorr(tiny, 0.031, -0.017)
    Dp = orc.decorr(tiny, 0.031, -0.017, sign=+1.0)
    assert np.max(np.abs(Dp - np.conj(D))) < 1e-15
    assert np.max(np.abs(D.imag)) > 1e-6     # the sign is observable


def test_decorr_gradient_matches_fd(tiny):
    l0, m0, h = 0.021, -0.013, 1e-7
    D, dl, dm = orc.decorr_with_grad(tiny, l0, m0)
    fl = (orc.decorr(tiny, l0 + h, m0) - orc.decorr(tiny, l0 - h, m0)) / (2 * h)
    fm = (orc.decorr(tiny, l0, m0 + h) - orc.decorr(tiny, l0, m0 - h)) / (2 * h)
    scale = max(np.max(np.abs(dl)), np.max(np.abs(dm)))
    assert np.max(np.abs(dl - fl)) < 1e-6 * scale
    assert np.max(np.abs(dm - fm)) < 1e-6 * scale


# ---------------------------------------------------------------- P
def effective_psf_closed_form(obs, src):
    # Section 2.2: the effective PSF is the inverse transform of the weighted
    # sampling function: both conjugate halves of a unit-weight delta give
    # 2 cos(2 pi (u l + v m)) at the bin centres, no decorrelation, no w.
    out = np.zeros((src.nl, src.nm))
    for k in range(obs.K):
        b, = np.nonzero(obs.bl_koff[1:] > k)[0][:1]
        nt, nc = obs.bl_bin[b]
        n_fb = -(-obs.n_ch // nc)
        T, F = divmod(k - obs.bl_koff[b], n_fb)
        ch = obs.freq_hz[F * nc:min(obs.n_ch, (F + 1) * nc)]
        u, v, _ = obs.uvw_c_m[obs.bl_tboff[b] + T] * ch.mean() / C
        for i in range(src.nl):
            li = src.l_first + i * src.dl
            mj = src.m_first + np.arange(src.nm) * src.dm
            out[i] += 2 * obs.W[k] * np.cos(2 * math.pi * (u * li + v * mj))
    return out


def test_phase_centre_patch_is_effective_psf(cfg1):
    obs, _ = cfg1
    src = ps.Source.centred(0.0, 0.0, 17, 20 * ps.ARCSEC)
    P = orc.patch_factored(obs, src)
    E = effective_psf_closed_form(obs, src)
    assert orc.peak_normalised_error(P, E)[0] < 1e-12


def test_peak_equals_sum_of_weighted_D(cfg1):
    obs, src = cfg1
    D = orc.decorr(obs, src.l0, src.m0)
    P = orc.patch_factored(obs, src, D)
    c = src.nl // 2
    peak = 2.0 * sum(float(obs.W[k]) * D[k].real for k in range(obs.K))
    assert abs(P[c, c] - peak) < 1e-12 * abs(peak)
    assert P[c, c] == pytest.approx(P.max(), rel=1e-12)


def test_normalised_patch(cfg1):
    """Row a6: the normalised PSF is 1 at the source pixel of a centred grid;
    on a grid that does not hold the source it equals the brute-force patch
    (explicit conjugate halves) divided by the brute-force value of a 1 x 1
    patch at the source; scaling every weight leaves it unchanged."""
    obs, src = cfg1
    N = orc.patch_normalised(obs, src)
    c = src.nl // 2
    assert abs(N[c, c] - 1.0) < 1e-12
    off = ps.Source(l0=src.l0, m0=src.m0, l_first=src.l0 + 40 * ps.ARCSEC, m_first=src.m0 - 25 * ps.ARCSEC,
                    dl=3 * ps.ARCSEC, dm=2 * ps.ARCSEC, nl=7, nm=5)
    at_src = ps.Source(l0=src.l0, m0=src.m0, l_first=src.l0, m_first=src.m0, dl=1.0, dm=1.0, nl=1, nm=1)
    ref = orc.patch_brute(obs, off).real / orc.patch_brute(obs, at_src).real[0, 0]
    assert np.max(np.abs(orc.patch_normalised(obs, off) - ref)) < 1e-12
    obs3 = ps.Observation(**{**obs.__dict__, "W": (3.0 * obs.W).astype(np.float32)})
    assert np.max(np.abs(orc.patch_normalised(obs3, off) - orc.patch_normalised(obs, off))) < 1e-13


def test_brute_force_with_explicit_conjugates(cfg1):
    obs, src = cfg1
    small = ps.Source.centred(src.l0, src.m0, 9, 7 * ps.ARCSEC, nm=11)
    Pb = orc.patch_brute(obs, small)
    P = orc.patch_factored(obs, small)
    assert np.max(np.abs(Pb.imag)) < 1e-13 * np.max(np.abs(Pb.real))
    assert orc.peak_normalised_error(Pb.real, P)[0] < 1e-12


def test_single_bin_closed_form():
    obs = ramp_observation(4, 4, 3.0, u0=(900.0, -2500.0, 310.0))
    l0, m0 = 0.013, 0.021
    src = ps.Source.centred(l0, m0, 5, 30 * ps.ARCSEC, nm=3)
    D = orc.decorr(obs, l0, m0)[0]
    n0 = math.sqrt(1 - l0 * l0 - m0 * m0)
    u, v, w = obs.uvw_c_m[0] * obs.freq_hz[0] / C
    P = orc.patch_factored(obs, src)
    for i in range(src.nl):
        for j in range(src.nm):
            x = i * src.dl + src.l_first - l0
            y = j * src.dm + src.m_first - m0
            th = 2 * math.pi * ((u - w * l0 / n0) * x + (v - w * m0 / n0) * y)
            want = 2 * (D.real * math.cos(th) - D.imag * math.sin(th))
            assert P[i, j] == pytest.approx(want, abs=1e-12)


def test_l_axis_is_first_index():
    # Only u varies and the w-shift vanishes (w = 0): P must vary along i (l)
    # and be constant along j (m) -- a swapped l/m grid fails this.
    obs = ramp_observation(6, 3, 2.0, u0=(1500.0, 0.0, 0.0))
    src = ps.Source.centred(0.004, 0.006, 7, 40 * ps.ARCSEC, nm=5)
    P = orc.patch_factored(obs, src)
    assert np.max(np.abs(P - P[:, :1])) < 1e-12 * np.max(np.abs(P))
    assert np.max(np.abs(P - P[:1, :])) > 1e-3 * np.max(np.abs(P))


def test_mirror_identity_of_sign_convention(tiny):
    # The literal "+" sign in both D and the imaging exponent gives the
    # point-mirrored patch of the paper's convention.
    src = ps.Source.centred(0.03, -0.02, 9, 25 * ps.ARCSEC)
    P = orc.patch_factored(tiny, src)
    Dp = orc.decorr(tiny, src.l0, src.m0, sign=+1.0)
    Pp = orc.patch_factored(tiny, src, D=Dp, sign=+1.0)
    # literal form == paper's patch at -x, -y (centred grid => index reversal)
    Pm = orc.patch_factored(tiny, src, D=np.conj(Dp), sign=-1.0)
    assert orc.peak_normalised_error(Pp, Pm)[0] < 1e-12
    assert orc.peak_normalised_error(Pm, P[::-1, ::-1])[0] < 1e-12
    assert orc.peak_normalised_error(P, P[::-1, ::-1])[0] > 1e-6


def test_linear_in_weights(tiny):
    src = ps.Source.centred(0.01, 0.02, 7, 20 * ps.ARCSEC)
    P1 = orc.patch_factored(tiny, src)
    t2 = ps.Observation(**{**tiny.__dict__, "W": (4.0 * tiny.W).astype(np.float32)})   # exact in float32
    P2 = orc.patch_factored(t2, src)
    assert orc.peak_normalised_error(P2, 4.0 * P1)[0] < 1e-14
    z = ps.Observation(**{**tiny.__dict__, "W": np.zeros_like(tiny.W)})
    assert np.all(orc.patch_factored(z, src) == 0.0)


def test_wshift_is_first_order_correct():
    # The linearised w-shift agrees with the exact w phase to second order in
    # the pixel offset.
    obs = ps.tiny_random(7, n_ant=5, n_t=4, n_ch=2, nt=2, nc=2, radius_m=20000.0)
    l0, m0 = 0.05, -0.04
    errs, errs_noshift = [], []
    for cell in (1e-7, 5e-8, 2.5e-8):           # patch well inside one fringe
        src = ps.Source.centred(l0, m0, 5, cell)
        D = orc.decorr(obs, l0, m0)
        Pw = orc.patch_fullw(obs, src, D)
        P = orc.patch_factored(obs, src, D)
        errs.append(np.max(np.abs(P - Pw)))
        # no shift: u' = u is the linearisation about the phase centre instead
        uk = orc.bin_centres_lambda(obs)
        x, y = orc.pixel_offsets(src)
        c = obs.W * D
        P0 = 2 * np.real(np.einsum("k,ki,kj->ij", c, np.exp(2j * np.pi * uk[:, 0, None] * x),
                                   np.exp(2j * np.pi * uk[:, 1, None] * y)))
        errs_noshift.append(np.max(np.abs(P0 - Pw)))
    # second order or better in the offset (the real part of the lowest term
    # can cancel between conjugate halves), and far below the error left when
    # the shift is dropped
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5
    assert all(e < 0.05 * e0 for e, e0 in zip(errs, errs_noshift))


def test_patch_pixels_agree_with_full_patch(cfg1):
    obs, src = cfg1
    P = orc.patch_factored(obs, src)
    ii, jj = [0, 32, 64, 10], [0, 32, 17, 64]
    vals = orc.patch_pixels(obs, src, ii, jj)
    assert np.max(np.abs(vals - P[ii, jj])) < 1e-12 * np.max(np.abs(P))


def test_ragged_and_bda_bins_brute_vs_factored():
    obs = ps.tiny_random(11, n_ant=5, n_t=11, n_ch=5, nt=4, nc=3, bda=True)
    assert len(set(map(tuple, obs.bl_bin))) > 1
    src = ps.Source.centred(0.02, 0.01, 5, 15 * ps.ARCSEC, nm=4)
    Pb = orc.patch_brute(obs, src)
    P = orc.patch_factored(obs, src)
    assert np.max(np.abs(Pb.imag)) < 1e-12 * np.max(np.abs(P))
    assert orc.peak_normalised_error(Pb.real, P)[0] < 1e-12


# ---------------------------------------------------------------- gradient
def _grad_setup(n_src=3, seed=0):
    obs = ps.tiny_random(21, n_ant=5, n_t=9, n_ch=4, nt=3, nc=2, radius_m=5000.0)
    g = np.random.default_rng(seed)
    srcs, fl, tg = [], [], []
    for _ in range(n_src):
        l0, m0 = g.uniform(-0.03, 0.03, 2)
        s = ps.Source.centred(l0, m0, 9, 10 * ps.ARCSEC, nm=7)
        f = 10 ** g.uniform(-1, 0)
        moved = s.with_direction(l0 + g.normal(0, 2 * ps.ARCSEC), m0 + g.normal(0, 2 * ps.ARCSEC))
        srcs.append(s)
        fl.append(f)
        tg.append(f * orc.patch_factored(obs, moved))
    return obs, srcs, np.array(fl), tg


def test_gradient_matches_central_differences():
    obs, srcs, fl, tg = _grad_setup()
    L, g_lm, g_f = orc.loss_grad_analytic(obs, srcs, fl, tg)
    fd = orc.loss_grad_fd(obs, srcs, fl, tg)
    assert L == pytest.approx(orc.loss_value(obs, srcs, fl, tg), rel=1e-12)
    assert np.max(np.abs(g_lm - fd)) < 1e-6 * np.max(np.abs(fd))
    # flux gradient: d/df sum (fP - T)^2 = 2 sum (fP - T) P, checked by FD in f
    h = 1e-6
    for n in range(len(srcs)):
        fp, fm = fl.copy(), fl.copy()
        fp[n] += h
        fm[n] -= h
        fdf = (orc.loss_value(obs, srcs, fp, tg) - orc.loss_value(obs, srcs, fm, tg)) / (2 * h)
        assert g_f[n] == pytest.approx(fdf, rel=1e-6)


def test_gradient_zero_at_generating_parameters():
    obs, srcs, fl, _ = _grad_setup(seed=1)
    tg = [f * orc.patch_factored(obs, s) for s, f in zip(srcs, fl)]
    L, g_lm, g_f = orc.loss_grad_analytic(obs, srcs, fl, tg)
    assert L < 1e-20
    assert np.max(np.abs(g_lm)) < 1e-6 and np.max(np.abs(g_f)) < 1e-9


# ---------------------------------------------------------------- properties
def test_random_tiny_observations_brute_vs_factored():
    hyp = pytest.importorskip("hypothesis")
    st = hyp.strategies

    @hyp.settings(max_examples=12, deadline=None, derandomize=True)
    @hyp.given(seed=st.integers(0, 10_000), nt=st.integers(1, 4), nc=st.integers(1, 3),
               l0=st.floats(-0.05, 0.05), m0=st.floats(-0.05, 0.05))
    def check(seed, nt, nc, l0, m0):
        obs = ps.tiny_random(seed, n_ant=3, n_t=5, n_ch=3, nt=nt, nc=nc)
        src = ps.Source.centred(l0, m0, 3, 30 * ps.ARCSEC, nm=4)
        Pb = orc.patch_brute(obs, src)
        P = orc.patch_factored(obs, src)
        assert np.max(np.abs(Pb.imag)) < 1e-12 * max(1.0, np.max(np.abs(P)))
        assert np.max(np.abs(Pb.real - P)) < 1e-12 * max(1.0, np.max(np.abs(P)))

    check()


# ---------------------------------------------------------------- Method 1 (sinc) decorrelation
def _boxcar_average(phase_of, a, b, m=200001):
    """Mean of exp(-2 pi i phase(x)) over [a, b] by the midpoint rule with m
    points (a plain quadrature of the continuous average)."""
    x = a + (np.arange(m) + 0.5) * (b - a) / m
    return np.mean(np.exp(-2j * np.pi * phase_of(x)))


def test_sinc_method_is_one_at_phase_centre(cfg1):
    obs, _ = cfg1
    assert np.array_equal(orc.decorr_sinc(obs, 0.0, 0.0), np.ones(obs.K))


@pytest.mark.parametrize("bin_len,g", [(8, 40.0), (20, 25.0), (5, 300.0)])
def test_sinc_method_is_continuous_average_of_linear_time_ramp(bin_len, g):
    """Method 1 [section 3.1] is the continuous average of the phase over the
    bin's time interval; on a track linear in time (one channel) it must equal
    the quadrature of that average over the interval covered by the bin's
    samples (n samples of spacing 1, centred on the bin centre)."""
    nu, l0 = 1.4e9, 0.02
    obs = ramp_observation(40, bin_len, g, nu=nu)
    Dh = orc.decorr_sinc(obs, l0, 0.0)
    for k in range(obs.K):
        n = min(40, (k + 1) * bin_len) - k * bin_len
        slope = g * nu / C * l0                      # turns per sample
        avg = _boxcar_average(lambda x: slope * x, -0.5 * n, 0.5 * n)
        assert abs(avg.imag) < 1e-9
        assert abs(Dh[k] - avg.real) < 1e-9, (k, Dh[k], avg)


def test_sinc_method_is_continuous_average_over_frequency():
    """One time sample, 6 channels of spacing dnu per bin: the frequency sinc
    is the average of exp(-2 pi i u nu l0 / c) over the bin's band n dnu
    relative to its centre frequency."""
    dnu, l0, n_ch = 4e6, 0.03, 12
    obs = ramp_observation(1, 1, 0.0, nu=1.4e9, n_ch=n_ch, bin_ch=6, dnu=dnu, u0=(5000.0, 1200.0, 10.0))
    Dh = orc.decorr_sinc(obs, l0, 0.0)
    u_m = 5000.0
    for k in range(obs.K):
        avg = _boxcar_average(lambda x: u_m * x / C * l0, -3 * dnu, 3 * dnu)
        assert abs(Dh[k] - avg.real) < 1e-9, (k, Dh[k], avg)


def test_sinc_method_real_bounded_and_close_to_exact_on_tracks(cfg1):
    """On Earth-rotation tracks Method 1 is real, at most 1 in magnitude, and
    differs from the exact discrete mean only by the curvature of the track,
    the discrete-versus-continuous gap and the dropped w term (small on
    these 30-sample, 1-channel bins at 0.58 deg)."""
    obs, src = cfg1
    Dh = orc.decorr_sinc(obs, src.l0, src.m0)
    D = orc.decorr(obs, src.l0, src.m0)
    assert np.all(np.abs(Dh) <= 1.0)
    assert np.max(np.abs(Dh - D.real)) < 5e-4
    assert np.max(np.abs(Dh - D.real)) > 1e-7   # an approximation, not the same quantity


# ---------------------------------------------------------------- Hogbom CLEAN [Algorithm 2]
def _image_grid(n=33, cell=2.0 * ps.ARCSEC, centre=(0.004, -0.003)):
    return ps.Source.centred(centre[0], centre[1], n, cell)


@pytest.mark.parametrize("gain", [1.0, 0.3])
def test_clean_single_source_residual_is_geometric(cfg1, gain):
    """A dirty image that is one distorted PSF (source on a pixel centre): each
    cycle finds the same pixel and removes the fraction gain of what is
    left, so after n cycles the residual is (1 - gain)^n of the dirty image
    and the components sum to (1 - (1 - gain)^n) of its peak."""
    obs, _ = cfg1
    grid = _image_grid()
    i0, j0 = 20, 11
    src = grid.with_direction(grid.l_first + i0 * grid.dl, grid.m_first + j0 * grid.dm)
    dirty = 0.7 * orc.patch_factored(obs, src)
    n = 1 if gain == 1.0 else 6
    res, comps = orc.hogbom_clean(obs, grid, dirty, gain, n)
    assert [(i, j) for i, j, _ in comps] == [(i0, j0)] * n
    assert np.max(np.abs(res - (1 - gain) ** n * dirty)) <= 1e-12 * np.max(np.abs(dirty))
    assert abs(sum(a for _, _, a in comps) - (1 - (1 - gain) ** n) * dirty[i0, j0]) <= 1e-12 * dirty[i0, j0]


def test_clean_two_sources_recovers_positions(cfg1):
    """Two sources of different flux on pixel centres, far enough apart that
    their PSFs barely overlap at the peaks: the brighter is found first and
    both positions appear among the components."""
    obs, _ = cfg1
    grid = _image_grid(n=65)
    pos = [(10, 12, 1.0), (50, 44, 0.45)]
    dirty = sum(f * orc.patch_factored(obs, grid.with_direction(grid.l_first + i * grid.dl,
                                                                grid.m_first + j * grid.dm))
                for i, j, f in pos)
    res, comps = orc.hogbom_clean(obs, grid, dirty, 0.5, 12)
    assert comps[0][:2] == (10, 12)
    found = {(i, j) for i, j, _ in comps}
    assert (10, 12) in found and (50, 44) in found
    assert np.max(np.abs(res)) < 0.2 * np.max(np.abs(dirty))


# ---------------------------------------------------------------- windowed averaging
def _with_windows(obs, win_t=None, win_c=None):
    return ps.Observation(**{**obs.__dict__, "win_t": win_t, "win_c": win_c})


def _triangle(m, n_bins):
    """Weights 1, 2, .., m, .., 2, 1 over each bin of 2m - 1 samples."""
    one = np.minimum(np.arange(1, 2 * m), np.arange(2 * m - 1, 0, -1)).astype(np.float32)
    return np.tile(one, n_bins)[None, :]


@pytest.mark.parametrize("m,d", [(2, 0.11), (4, 0.07), (6, 0.23), (9, 0.031)])
def test_triangle_time_window_is_squared_dirichlet(m, d):
    """The triangle of 2m - 1 samples is the convolution of two m-sample
    boxcars, so on a linear phase ramp (step d turns per sample, bin centre
    on the middle sample) its normalised transform is the square of the
    m-sample Dirichlet kernel."""
    nu, l0 = 1.4e9, 0.01
    n = 2 * m - 1
    obs = _with_windows(ramp_observation(3 * n, n, d * C / (nu * l0), nu=nu, axis=0), win_t=_triangle(m, 3))
    D = orc.decorr(obs, l0, 0.0)
    assert np.allclose(D, dirichlet(m, d) ** 2, atol=1e-12, rtol=0)
    box = orc.decorr(_with_windows(obs), l0, 0.0)
    assert np.max(np.abs(D - box)) > 1e-3          # the window is observable


@pytest.mark.parametrize("m", [3, 5])
def test_triangle_channel_window_is_squared_dirichlet(m):
    nu, m0, dnu = 1.4e9, -0.02, 5e6
    n = 2 * m - 1
    obs = ramp_observation(2, 1, 0.0, nu=nu, n_ch=2 * n, bin_ch=n, dnu=dnu, u0=(300.0, 2100.0, 0.0))
    obs = _with_windows(obs, win_c=_triangle(m, 2))
    D = orc.decorr(obs, 0.0, m0)
    assert np.allclose(D, dirichlet(m, 2100.0 * dnu * m0 / C) ** 2, atol=1e-12, rtol=0)


def test_window_of_ones_is_boxcar_and_scale_free(tiny):
    l0, m0 = 0.031, -0.017
    box = orc.decorr(tiny, l0, m0)
    ones = _with_windows(tiny, np.ones((tiny.n_bl, tiny.n_t), np.float32),
                         np.ones((tiny.n_bl, tiny.n_ch), np.float32))
    assert np.max(np.abs(orc.decorr(ones, l0, m0) - box)) < 1e-15
    win = ps.tapered_windows(tiny)
    Dw = orc.decorr(win, l0, m0)
    scaled = _with_windows(win, (4.0 * win.win_t).astype(np.float32), (0.25 * win.win_c).astype(np.float32))
    assert np.max(np.abs(orc.decorr(scaled, l0, m0) - Dw)) < 1e-15     # power-of-two scales: exact in float32
    assert np.max(np.abs(Dw - box)) > 1e-4


def test_delta_window_on_the_bin_centre_sample_gives_one():
    """A window that keeps only each bin's middle sample (whose uvw is the bin
    centre) has no smearing: D = 1 at any direction."""
    n = 7
    obs = ramp_observation(3 * n, n, 40.0, axis=1)
    wt = np.zeros((1, 3 * n), np.float32)
    wt[0, n // 2::n] = 2.0
    D = orc.decorr(_with_windows(obs, win_t=wt), 0.02, -0.05)
    assert np.all(D == 1.0)


def test_zero_window_bin_has_zero_D_and_others_unchanged(tiny):
    win = ps.tapered_windows(tiny)
    tab = orc.bin_table(tiny)
    k = 5
    b, t0, t1 = int(tab.b[k]), int(tab.t0[k]), int(tab.t1[k])
    wt = win.win_t.copy()
    wt[b, t0:t1] = 0.0                      # every bin of baseline b in this time bin
    z = _with_windows(win, wt, win.win_c)
    Dz, Dw = orc.decorr(z, 0.03, 0.01), orc.decorr(win, 0.03, 0.01)
    hit = (tab.b == b) & (tab.t0 == t0)
    assert np.all(Dz[hit] == 0.0)
    assert np.array_equal(Dz[~hit], Dw[~hit])


def test_windowed_decorr_matches_explicit_loops():
    obs = ps.tapered_windows(ps.tiny_random(4, n_ant=5, n_t=11, n_ch=7, nt=4, nc=3, bda=True), strength=0.8)
    D = orc.decorr(obs, 0.027, 0.011)
    Db = orc.decorr_brute(obs, 0.027, 0.011)
    assert np.max(np.abs(D - Db)) < 1e-12


def test_windowed_decorr_gradient_matches_fd():
    obs = ps.tapered_windows(ps.tiny_random(2, n_t=9, n_ch=5, nt=3, nc=2))
    l0, m0, h = 0.021, -0.013, 1e-7
    D, dl, dm = orc.decorr_with_grad(obs, l0, m0)
    assert np.max(np.abs(D - orc.decorr(obs, l0, m0))) < 1e-15
    fl = (orc.decorr(obs, l0 + h, m0) - orc.decorr(obs, l0 - h, m0)) / (2 * h)
    fm = (orc.decorr(obs, l0, m0 + h) - orc.decorr(obs, l0, m0 - h)) / (2 * h)
    scale = max(np.max(np.abs(dl)), np.max(np.abs(dm)))
    assert np.max(np.abs(dl - fl)) < 1e-6 * scale
    assert np.max(np.abs(dm - fm)) < 1e-6 * scale


def test_method1_rejects_windows(tiny):
    with pytest.raises(ValueError):
        orc.decorr_sinc(ps.tapered_windows(tiny), 0.01, 0.0)


# ---------------------------------------------------------------- full-w patch
def _fullw_by_imaging(obs, src):
    """Brute force by another route: simulate each sample's visibility of a
    unit point source at (l0, m0) with the full w-term, average the samples
    of every bin, then image the averaged visibilities (both conjugate
    halves) at each pixel with the full w-term in absolute coordinates.
    No decorrelation factor, no offsets, no linearisation."""
    tab = orc.bin_table(obs)
    n0 = math.sqrt(1.0 - src.l0 ** 2 - src.m0 ** 2)
    li = src.l_first + np.arange(src.nl) * src.dl
    mj = src.m_first + np.arange(src.nm) * src.dm
    out = np.zeros((src.nl, src.nm))
    for k in range(len(tab.b)):
        b = int(tab.b[k])
        chans = range(int(tab.c0[k]), int(tab.c1[k]))
        vis, n = 0j, 0
        for t in range(int(tab.t0[k]), int(tab.t1[k])):
            for c in chans:
                u, v, w = obs.uvw_m[b, t] * obs.freq_hz[c] / C
                vis += np.exp(-2j * math.pi * (u * src.l0 + v * src.m0 + w * (n0 - 1.0)))
                n += 1
        vis /= n
        nu = sum(obs.freq_hz[c] for c in chans) / len(chans)
        uk, vk, wk = obs.uvw_c_m[int(tab.tb[k])] * nu / C
        for i, l in enumerate(li):
            nn = np.sqrt(1.0 - l * l - mj ** 2)
            out[i] += 2.0 * float(obs.W[k]) * np.real(vis * np.exp(2j * math.pi * (uk * l + vk * mj + wk * (nn - 1.0))))
    return out


@pytest.mark.parametrize("l0,m0", [(0.03, -0.02), (-0.2, 0.15)])
def test_fullw_patch_equals_simulate_average_image(l0, m0):
    obs = ps.tiny_random(6, n_ant=4, n_t=6, n_ch=3, nt=3, nc=2, radius_m=15000.0)
    src = ps.Source.centred(l0, m0, 9, 20.0 * ps.ARCSEC, nm=7)
    ref = _fullw_by_imaging(obs, src)
    P = orc.patch_fullw(obs, src)
    assert orc.peak_normalised_error(P, ref)[0] < 1e-11
    # the linearised patch differs visibly at this patch size and baseline length
    assert orc.peak_normalised_error(orc.patch_factored(obs, src), ref)[0] > 1e-6


def test_fullw_patch_without_w_is_the_linearised_patch():
    obs = ps.tiny_random(6, n_ant=4, n_t=6, n_ch=3, nt=3, nc=2, radius_m=15000.0)
    flat = ps.Observation(**{**obs.__dict__, "uvw_m": obs.uvw_m * np.array([1.0, 1.0, 0.0]),
                             "uvw_c_m": obs.uvw_c_m * np.array([1.0, 1.0, 0.0])})
    src = ps.Source.centred(0.1, -0.05, 11, 30.0 * ps.ARCSEC)
    assert orc.peak_normalised_error(orc.patch_fullw(flat, src), orc.patch_factored(flat, src))[0] < 1e-12


def test_fullw_peak_and_pixels(cfg1):
    obs, src = cfg1
    src = src.with_direction(src.l0, src.m0)
    P = orc.patch_fullw(obs, src)
    c = src.nl // 2
    D = orc.decorr(obs, src.l0, src.m0)
    assert abs(P[c, c] - 2.0 * np.sum(obs.W * D.real)) < 1e-9 * abs(P[c, c])
    ii, jj = np.array([0, 3, c, src.nl - 1]), np.array([5, 0, c, src.nm - 2])
    assert np.max(np.abs(orc.patch_fullw_pixels(obs, src, ii, jj) - P[ii, jj])) < 1e-9 * abs(P[c, c])


# ---------------------------------------------------------------- Method 2
def _one_visibility(u, v, W=1.0):
    """One baseline, one sample, one channel at nu = c (so metres are
    wavelengths exactly), w = 0."""
    uvw = np.array([[[u, v, 0.0]]])
    bl_bin = np.array([[1, 1]], np.int32)
    koff, tboff = ps.bin_tables(1, 1, bl_bin)
    return ps.Observation(ant_enu=np.zeros((2, 3)), bl_ant=np.array([[0, 1]], np.int32), times_s=np.zeros(1),
                          uvw_m=uvw, freq_hz=np.array([C]), bl_bin=bl_bin, bl_koff=koff, bl_tboff=tboff,
                          uvw_c_m=uvw[0].copy(), W=np.array([W], np.float32))


def test_method2_at_phase_centre_is_the_effective_psf(cfg1):
    obs, _ = cfg1
    P = orc.method2_effective_psf(obs, 64, 4.0 * ps.ARCSEC)
    Q = orc.method2_patch(P, 4.0 * ps.ARCSEC, 0.0, 0.0, 30.0, 2e6, 1.4e9)
    assert np.max(np.abs(P - Q)) < 1e-12 * np.max(np.abs(P))
    assert P[32, 32] == pytest.approx(2.0 * float(np.sum(obs.W, dtype=np.float64)), rel=1e-12)


@pytest.mark.parametrize("a,b", [(3, -5), (0, 7), (-11, 2)])
def test_method2_grid_aligned_visibility_is_scaled_by_dhat(a, b):
    """A visibility on a uv cell: its effective PSF is periodic on the grid,
    its spectrum two spikes at +-(a, b), so Method 2 returns the effective
    PSF times D^ of that cell (which cell the spectrum lands on and how the
    grid is centred are what this checks)."""
    N, cell = 32, 1e-3
    du = 1.0 / (N * cell)
    obs = _one_visibility(a * du, b * du, W=0.7)
    P = orc.method2_effective_psf(obs, N, cell)
    l0, m0, dt, dnu, nu = 0.02, -0.015, 3000.0, 4e7, 1.0e9
    Q = orc.method2_patch(P, cell, l0, m0, dt, dnu, nu)
    d = orc.method2_dhat(a * du, b * du, l0, m0, dt, dnu, nu)
    assert 0.01 < abs(d) < 0.999
    assert np.max(np.abs(Q - d * P)) < 1e-12


def test_method2_fringe_rate_matches_a_polar_circular_track():
    """At the celestial pole a baseline's uv track is a circle turning at
    omega_E: the model's time smearing phase equals the exact change of
    u.l0 across a bin of dt seconds (to (omega dt)^2)."""
    g = np.random.default_rng(3)
    bl = g.normal(0.0, 3000.0, size=(4, 3))
    nu, dt = 1.4e9, 20.0
    for t in (-3000.0, 0.0, 1234.0):
        H = ps.OMEGA_EARTH * np.array([t - dt / 2, t, t + dt / 2])
        uvw = ps.uvw_tracks(bl, H, lat=math.radians(52.0), dec=math.radians(90.0)) * nu / C   # [bl, 3, 3]
        for l0, m0 in ((0.03, -0.01), (-0.02, 0.05)):
            exact = 2 * math.pi * ((uvw[:, 2, 0] - uvw[:, 0, 0]) * l0 + (uvw[:, 2, 1] - uvw[:, 0, 1]) * m0)
            u0, v0 = uvw[:, 1, 0], uvw[:, 1, 1]
            model = 2 * math.pi * orc.OMEGA_EARTH * (-v0 * l0 + u0 * m0) * dt
            assert np.allclose(model, exact, rtol=1e-6, atol=0)
            d = orc.method2_dhat(u0, v0, l0, m0, dt, 0.0, nu)
            assert np.allclose(d, np.sinc(exact / (2 * math.pi)), rtol=0, atol=1e-6)


def test_method2_frequency_term_is_the_band_average_along_the_baseline():
    """For a direction along the baseline the model's bandwidth phase is the
    exact one: D^ (no time smearing) equals the band average of the fringe
    over dnu, by quadrature."""
    u0, v0 = 1800.0, -2400.0                   # wavelengths at nu
    nu, dnu = 1.4e9, 3e6
    unit = np.array([u0, v0]) / math.hypot(u0, v0)
    for r in (0.01, 0.04):
        l0, m0 = r * unit
        f = nu + dnu * ((np.arange(200000) + 0.5) / 200000 - 0.5)       # midpoint rule
        avg = np.mean(np.exp(-2j * math.pi * (u0 * l0 + v0 * m0) * f / nu))
        d = orc.method2_dhat(u0, v0, l0, m0, 0.0, dnu, nu)
        assert abs(abs(avg) - d) < 1e-8


def test_method2_on_grid_visibilities_equals_direct_sum():
    """Several visibilities on uv cells of the grid: Method 2 equals the
    direct sum 2 sum_k W_k D^(u_k) cos(2 pi (u_k x + v_k y)) over the patch,
    each visibility scaled by the D^ of its own cell."""
    N, cell = 64, 2e-4
    du = 1.0 / (N * cell)
    cells = [(3, -5), (0, 7), (-11, 2), (20, 13), (-7, -29)]
    W = [0.7, 1.3, 0.4, 1.0, 0.9]
    uvw = np.array([[[a * du, b * du, 0.0]] for a, b in cells])
    bl_bin = np.ones((len(cells), 2), np.int32)
    koff, tboff = ps.bin_tables(1, 1, bl_bin)
    obs = ps.Observation(ant_enu=np.zeros((2, 3)), bl_ant=np.zeros((len(cells), 2), np.int32),
                         times_s=np.zeros(1), uvw_m=uvw, freq_hz=np.array([C]), bl_bin=bl_bin, bl_koff=koff,
                         bl_tboff=tboff, uvw_c_m=uvw[:, 0, :].copy(), W=np.array(W, np.float32))
    l0, m0, dt, dnu, nu = 0.05, 0.03, 4000.0, 3e7, 1.0e9
    Q = orc.method2_patch(orc.method2_effective_psf(obs, N, cell), cell, l0, m0, dt, dnu, nu)
    x, _ = orc.method2_grid(N, cell)
    X, Y = np.meshgrid(x, x, indexing="ij")
    ref = np.zeros((N, N))
    for (a, b), w in zip(cells, W):
        d = orc.method2_dhat(a * du, b * du, l0, m0, dt, dnu, nu)
        ref += 2.0 * float(np.float32(w)) * d * np.cos(2 * math.pi * (a * du * X + b * du * Y))
    assert np.max(np.abs(Q - ref)) < 1e-11 * np.max(np.abs(ref))
    assert np.max(np.abs(Q - orc.method2_effective_psf(obs, N, cell))) > 0.1 * np.max(np.abs(ref))


# ---------------------------------------------------------------- CLEAN with Method-2 PSFs
def _placed(Q, i, j, nl, nm):
    """Q (centred N x N) with its centre on image pixel (i, j); outside 0."""
    N = Q.shape[0]
    out = np.zeros((nl, nm))
    for a in range(nl):
        for b in range(nm):
            u, v = a - i + N // 2, b - j + N // 2
            if 0 <= u < N and 0 <= v < N:
                out[a, b] = Q[u, v]
    return out


@pytest.mark.parametrize("pix", [(20, 11), (2, 30)])
def test_method2_clean_single_source_residual_is_geometric(cfg1, pix):
    """A dirty image that is one Method-2 PSF laid on a pixel (near the edge
    too, where the PSF is cut): every cycle finds that pixel and removes the
    fraction gain of what is left."""
    obs, _ = cfg1
    grid = _image_grid()
    N, cell = 32, grid.dl
    Peff = orc.method2_effective_psf(obs, N, cell)
    i0, j0 = pix
    l0, m0 = grid.l_first + i0 * grid.dl, grid.m_first + j0 * grid.dm
    Q = orc.method2_patch(Peff, cell, l0, m0, 30.0, 1e6, 1.4e9)
    dirty = 0.7 * _placed(Q, i0, j0, grid.nl, grid.nm)
    gain, n = 0.3, 6
    res, comps = orc.hogbom_clean_method2(Peff, grid, dirty, gain, n, 30.0, 1e6, 1.4e9)
    assert [(i, j) for i, j, _ in comps] == [(i0, j0)] * n
    assert np.max(np.abs(res - (1 - gain) ** n * dirty)) < 1e-12 * np.max(np.abs(dirty))
    assert abs(sum(a for _, _, a in comps) - (1 - (1 - gain) ** n) * dirty[i0, j0]) < 1e-12 * abs(dirty[i0, j0])


def test_method2_clean_at_the_phase_centre_uses_the_effective_psf(cfg1):
    """At the pixel of the phase centre D^ = 1, so the subtracted PSF is the
    effective PSF itself."""
    obs, _ = cfg1
    grid = ps.Source.centred(0.0, 0.0, 33, 4.0 * ps.ARCSEC)
    N = 64
    Peff = orc.method2_effective_psf(obs, N, grid.dl)
    dirty = _placed(Peff, 16, 16, 33, 33)
    res, comps = orc.hogbom_clean_method2(Peff, grid, dirty, 1.0, 1, 30.0, 1e6, 1.4e9)
    assert comps[0][:2] == (16, 16)
    assert np.max(np.abs(res)) < 1e-12 * np.max(np.abs(dirty))


def test_empty_observation_gives_empty_sums():
    """No baselines: no bins, no factors, a zero patch (empty sums)."""
    obs = ps.Observation(ant_enu=np.zeros((2, 3)), bl_ant=np.zeros((0, 2), np.int32), times_s=np.zeros(4),
                         uvw_m=np.zeros((0, 4, 3)), freq_hz=np.array([1.4e9]), bl_bin=np.zeros((0, 2), np.int32),
                         bl_koff=np.zeros(1, np.int64), bl_tboff=np.zeros(1, np.int64), uvw_c_m=np.zeros((0, 3)),
                         W=np.zeros(0, np.float32))
    src = ps.Source.centred(0.01, -0.02, 9, 2.0 * ps.ARCSEC)
    assert orc.decorr(obs, 0.01, -0.02).shape == (0,)
    assert np.all(orc.patch_factored(obs, src) == 0.0)
    assert np.all(orc.patch_fullw(obs, src) == 0.0)
