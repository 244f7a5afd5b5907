"""GPU parity on bins wider than one register chunk of channels (19 and 18
channels per bin, with a ragged last bin per baseline): the decorrelation
factors (boxcar and windowed), the patch, and the adjoint's gradient against
the FP64 oracle.  Bars: D within 2e-6, patches 1e-5 of the peak, gradients
1e-4.  D is checked on a 200 MHz band where the bins decorrelate strongly;
the patches on a 40 MHz band (mean |D| about 0.84) and a 100 MHz band (the
peak a small fraction of the sum of the term sizes, where split-BF16's
per-term rounding of about 2^-17 of a term averages least), the gradients
on the 40 MHz band."""
import numpy as np
import pytest

import oracle as orc
import psf_synth as ps

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2009_07010_amd as pk
    pk.lib()
    return pk


def _obs(windowed, nu_lo=1.3e9, nu_hi=1.5e9, n_ant=6):
    obs = ps.tiny_random(41, n_ant=n_ant, n_t=12, n_ch=37, nt=3, nc=19, radius_m=4000.0, nu_lo=nu_lo, nu_hi=nu_hi)
    return ps.tapered_windows(obs, strength=0.8) if windowed else obs


@pytest.mark.parametrize("windowed", [False, True])
def test_wide_bin_decorr(pk, windowed):
    obs = _obs(windowed)
    assert int(obs.bl_bin[0][1]) == 19 and len(obs.freq_hz) == 37  # bins of 19 and 18 channels
    dobs = pk.DeviceObservation(obs)
    for l0, m0 in ((0.002, -0.001), (-0.04, 0.03)):
        Dg = pk.decorr(dobs, l0, m0).cpu().numpy().astype(np.complex128)
        D = orc.decorr(obs, l0, m0)
        print(f"wide bins windowed={windowed} D: {np.max(np.abs(Dg - D)):.2e}", flush=True)
        assert np.max(np.abs(Dg - D)) < 2e-6
        assert np.max(np.abs(D - 1.0)) > 1e-3  # the bins do decorrelate


@pytest.mark.parametrize("windowed", [False, True])
@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
@pytest.mark.parametrize("band,n_ant", [((1.38e9, 1.42e9), 6), ((1.35e9, 1.45e9), 6), ((1.35e9, 1.45e9), 10)])
def test_wide_bin_patch(pk, windowed, prec, band, n_ant):
    """40 MHz (mean |D| about 0.84) and 100 MHz bands (strong decorrelation:
    the peak is a small fraction of the sum of the term sizes), with 120 bins
    (below 256: split-BF16 requests run FP32 products) and 360 bins (split
    products)."""
    obs = _obs(windowed, band[0], band[1], n_ant)
    src = ps.Source.centred(0.0021, -0.0013, 33, 2.0 * ps.ARCSEC)
    D = orc.decorr(obs, src.l0, src.m0)
    P = orc.patch_factored(obs, src, D)
    Pg = pk.patch(pk.DeviceObservation(obs), src, prec=prec).double().cpu().numpy()
    err = orc.peak_normalised_error(Pg, P)[0]
    ratio = np.max(np.abs(P)) / (2.0 * np.sum(obs.W * np.abs(D)))
    print(f"wide bins {band[1] - band[0]:.0e} Hz K={obs.K} windowed={windowed} {prec}: {err:.2e} "
          f"(mean |D| {np.mean(np.abs(D)):.2f}, peak / sum of term sizes {ratio:.2f})", flush=True)
    assert err < TOL


@pytest.mark.parametrize("windowed", [False, True])
def test_wide_bin_gradient(pk, windowed):
    """dL/d(l0, m0, flux) of the patch-fitting loss through the gradient
    sums of D over two register chunks of channels and a partial one."""
    obs = _obs(windowed, 1.38e9, 1.42e9)
    cell = 2.0 * ps.ARCSEC
    srcs = [ps.Source.centred(l0, m0, 33, cell) for l0, m0 in ((0.0021, -0.0013), (-0.0017, 0.0009))]
    fluxes = [1.0, 0.4]
    g = np.random.default_rng(4)
    moved = [s.with_direction(s.l0 + g.normal(0, ps.ARCSEC), s.m0 + g.normal(0, ps.ARCSEC)) for s in srcs]
    T64 = [(f * orc.patch_factored(obs, m)).astype(np.float32).astype(np.float64) for f, m in zip(fluxes, moved)]
    L_ref, g_ref, gf_ref = orc.loss_grad_analytic(obs, srcs, fluxes, T64)
    P64 = [orc.patch_factored(obs, s) for s in srcs]
    fscale = [2.0 * np.sum(np.abs((f * P - t) * P)) for f, P, t in zip(fluxes, P64, T64)]
    dobs = pk.DeviceObservation(obs)
    lm = torch.tensor([[s.l0, s.m0] for s in srcs], dtype=torch.float64, requires_grad=True)
    f = torch.tensor(fluxes, dtype=torch.float32, device="cuda", requires_grad=True)
    out = pk.psf_patch_fn().apply(lm, f, dobs, srcs, "split_bf16")
    loss = ((out.double() - torch.as_tensor(np.stack(T64), device="cuda")) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert abs(float(loss.detach()) - L_ref) <= 1e-3 * L_ref
    g_lm, g_f = lm.grad.numpy(), f.grad.double().cpu().numpy()
    for s in range(len(srcs)):
        err = np.max(np.abs(g_lm[s] - g_ref[s])) / np.max(np.abs(g_ref[s]))
        ferr = abs(g_f[s] - gf_ref[s]) / fscale[s]
        print(f"wide bins windowed={windowed} grad src{s}: dir {err:.2e} flux {ferr:.2e}", flush=True)
        assert err <= 1e-4 and ferr <= 1e-4


def test_wide_bin_batched(pk):
    """The batched path forms its records with the several-source launch of
    the decorrelation: mixed patch sizes on the wide bins, windowed."""
    obs = _obs(True, 1.38e9, 1.42e9)
    cell = 2.0 * ps.ARCSEC
    srcs = [ps.Source.centred(l0, m0, n, cell)
            for l0, m0, n in ((0.0021, -0.0013, 65), (-0.0017, 0.0009, 33), (0.0004, 0.0019, 129))]
    parts = pk.split_patches(pk.patch_batched(pk.DeviceObservation(obs), srcs, prec="split_bf16"), srcs)
    torch.cuda.synchronize()
    for s, P in zip(srcs, parts):
        err = orc.peak_normalised_error(P.double().cpu().numpy(), orc.patch_factored(obs, s))[0]
        print(f"wide bins batched {s.nl}: {err:.2e}", flush=True)
        assert err < TOL


def _long_bins(windowed, uneven=False):
    """Few bins of many samples (60 x 16 = 960, or per-baseline bins of 7 to
    60 samples by 3 to 16 channels with short last bins): too few bins to
    fill the GPU with one lane each, so the decorrelation takes one wave per
    bin (lane-strided samples, fixed butterfly reduction)."""
    if uneven:
        g = np.random.default_rng(44)
        ants = ps.layout_disc(6, 3000.0, g)
        bins = np.stack([g.integers(7, 61, 15), g.integers(3, 17, 15)], axis=1)
        obs = ps.make_observation(ants, 600, 1.0, ps.channel_centres(1.3e9, 1.5e9, 64), bins,
                                  weight_rng=np.random.default_rng(45))
    else:
        obs = ps.tiny_random(43, n_ant=6, n_t=600, n_ch=64, nt=60, nc=16, radius_m=3000.0, dt=1.0)
    assert obs.K < 512 * 64 and obs.n_bl * obs.n_t * obs.n_ch >= 64 * obs.K
    return ps.tapered_windows(obs, strength=0.8) if windowed else obs


@pytest.mark.parametrize("windowed", [False, True])
@pytest.mark.parametrize("uneven", [False, True])
def test_long_bins_decorr_patch_and_gradient(pk, windowed, uneven):
    obs = _long_bins(windowed, uneven)
    dobs = pk.DeviceObservation(obs)
    src = ps.Source.centred(0.004, -0.003, 65, 2.0 * ps.ARCSEC)
    D = orc.decorr(obs, src.l0, src.m0)
    Dg = pk.decorr(dobs, src.l0, src.m0).cpu().numpy().astype(np.complex128)
    print(f"long bins K={obs.K} uneven={uneven} windowed={windowed} D: {np.max(np.abs(Dg - D)):.2e} "
          f"(mean |D| {np.mean(np.abs(D)):.2f})", flush=True)
    assert np.max(np.abs(Dg - D)) < 2e-6
    P = orc.patch_factored(obs, src, D)
    for prec in ("fp32", "split_bf16"):
        err = orc.peak_normalised_error(pk.patch(dobs, src, prec=prec).double().cpu().numpy(), P)[0]
        print(f"long bins patch {prec}: {err:.2e}", flush=True)
        assert err < TOL
    moved = src.with_direction(src.l0 + ps.ARCSEC, src.m0 - 0.5 * ps.ARCSEC)
    T = orc.patch_factored(obs, moved)
    _, g_ref, _ = orc.loss_grad_analytic(obs, [src], [1.0], [T])
    G = torch.as_tensor(2.0 * (P - T), dtype=torch.float32, device="cuda").reshape(-1)
    got = pk.patch_backward(dobs, [src], G, "split_bf16").cpu().numpy()
    err = np.max(np.abs(got[0] - g_ref[0])) / np.max(np.abs(g_ref[0]))
    print(f"long bins gradient: {err:.2e}", flush=True)
    assert err <= 1e-4
