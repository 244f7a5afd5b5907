"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bar: peak-normalised max error <= 1e-5 for the FP32 and split forms (the
target error of the PSF patches), D_k within FP32 rounding of the oracle.
"""
import os

import numpy as np
import pytest

import oracle as orc
import psf_synth as ps

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2009_07010_amd as pk  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-5
ACCURATE = ["fp32", "split_bf16", "split_fp16"]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pk.lib()


@pytest.fixture(scope="module")
def cfg1():
    obs = ps.observation(1)
    src = ps.sources(1)[0]
    D = orc.decorr(obs, src.l0, src.m0)
    P = orc.patch_factored(obs, src, D)
    return obs, pk.DeviceObservation(obs), src, D, P


def gpu_patch(dobs, src, prec, D=None):
    P = pk.patch(dobs, src, prec=prec, D=D)
    torch.cuda.synchronize()
    return P.double().cpu().numpy()


def test_decorr_config1(cfg1):
    obs, dobs, src, D, _ = cfg1
    Dg = pk.decorr(dobs, src.l0, src.m0)
    torch.cuda.synchronize()
    Dg = Dg.cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(Dg - D)) < 2e-6


@pytest.mark.parametrize("prec", ACCURATE)
def test_patch_config1(cfg1, prec):
    obs, dobs, src, D, P = cfg1
    Pg = gpu_patch(dobs, src, prec)
    err, rms = orc.peak_normalised_error(Pg, P)
    print(f"config1 {prec}: max {err:.3e} rms {rms:.3e}")
    assert err < TOL


@pytest.mark.parametrize("prec", ACCURATE)
def test_patch_config1_given_D(cfg1, prec):
    obs, dobs, src, D, P = cfg1
    Dt = torch.as_tensor(D.astype(np.complex64)).cuda()
    Pg = gpu_patch(dobs, src, prec, D=Dt)
    assert orc.peak_normalised_error(Pg, P)[0] < TOL


def test_plain_bf16_negative_control(cfg1):
    # one BF16 product per term (no split) misses the bar at this size
    obs, dobs, src, D, P = cfg1
    Pg = gpu_patch(dobs, src, "plain_bf16")
    err = orc.peak_normalised_error(Pg, P)[0]
    print(f"config1 plain_bf16: max {err:.3e}")
    assert err > TOL


def test_config1_twenty_sample_bins():
    obs = ps.observation(1, bin_samples=20)
    assert obs.K == 630
    src = ps.sources(1)[0]
    P = orc.patch_factored(obs, src)
    dobs = pk.DeviceObservation(obs)
    for prec in ACCURATE:
        assert orc.peak_normalised_error(gpu_patch(dobs, src, prec), P)[0] < TOL


@pytest.mark.parametrize("n,nm", [(1, 1), (2, 3), (17, 17), (33, 16), (65, 129), (129, 129), (160, 161),
                                  (257, 257)])
def test_patch_sizes(n, nm):
    obs = ps.tiny_random(31, n_ant=6, n_t=40, n_ch=6, nt=7, nc=4, radius_m=4000.0)
    src = ps.Source.centred(0.012, -0.021, n, 1.5 * ps.ARCSEC, nm=nm)
    P = orc.patch_factored(obs, src)
    dobs = pk.DeviceObservation(obs)
    for prec in ACCURATE:
        err = orc.peak_normalised_error(gpu_patch(dobs, src, prec), P)[0]
        assert err < TOL, (prec, err)


def _grid(l0, m0, nl, nm, dl, dm, shift_l=0.0, shift_m=0.0):
    """A patch grid around (l0, m0) whose centre row sits shift_l pixels
    (and centre column shift_m pixels) away from the source."""
    return ps.Source(l0=l0, m0=m0, l_first=l0 - 0.5 * (nl - 1) * dl + shift_l * dl,
                     m_first=m0 - 0.5 * (nm - 1) * dm + shift_m * dm, dl=dl, dm=dm, nl=nl, nm=nm)


@pytest.mark.parametrize("nl,nm,dl,dm", [(65, 70, 2.0, 1.5), (129, 140, -1.5, 1.5), (129, 129, 1.5, 1.5),
                                         (257, 257, 1.5, 1.5), (257, 270, 1.0, -2.0)])
@pytest.mark.parametrize("shift_l,shift_m", [(0.0, 0.0), (0.37, -5.2), (-40.0, 3.0)])
def test_symmetric_form(nl, nm, dl, dm, shift_l, shift_m):
    """Patches 65, 129 or 257 rows high take the symmetric form of the
    contraction (cos and sin rows of the non-negative half of the row
    offsets, 32 visibilities per chunk): centred grids, grids whose centre
    row is a fraction of a pixel or many pixels off the source (the offset
    factor joins the coefficients), widths within the family, either sign
    of the cell; K = 1456 is not a multiple of the chunk."""
    obs = ps.tiny_random(37, n_ant=14, n_t=31, n_ch=5, nt=4, nc=3, radius_m=5000.0)
    assert obs.K % 32 != 0
    src = _grid(0.014, -0.019, nl, nm, dl * ps.ARCSEC, dm * ps.ARCSEC, shift_l, shift_m)
    P = orc.patch_factored(obs, src)
    dobs = pk.DeviceObservation(obs)
    for prec in ACCURATE:
        err = orc.peak_normalised_error(gpu_patch(dobs, src, prec), P)[0]
        print(f"symmetric {nl}x{nm} shift ({shift_l}, {shift_m}) {prec}: {err:.2e}", flush=True)
        assert err < TOL, (prec, err)


@pytest.mark.parametrize("n,nm", [(4096, 4096), (1, 4096), (4096, 1), (4096, 7)])
def test_patch_maximum_sizes(n, nm):
    """The largest patches the boundary accepts (4096 per side) and the
    thinnest, on a small observation (K = 180)."""
    obs = ps.tiny_random(33, n_ant=6, n_t=40, n_ch=6, nt=7, nc=4, radius_m=4000.0)
    src = ps.Source.centred(0.012, -0.021, n, 0.5 * ps.ARCSEC, nm=nm)
    P = orc.patch_factored(obs, src)
    dobs = pk.DeviceObservation(obs)
    for prec in ("fp32", "split_bf16"):
        err = orc.peak_normalised_error(gpu_patch(dobs, src, prec), P)[0]
        print(f"{n}x{nm} {prec}: {err:.2e}", flush=True)
        assert err < TOL, (prec, err)


def test_single_bin_observation():
    """K = 1: a single term, whose split-BF16 product alone would be off by
    up to 3 2^-16 of it; below 256 bins the library contracts split-BF16
    requests with FP32 products, so every precision meets 1e-5."""
    obs = ps.make_observation(np.array([[0.0, 0.0, 0.0], [1200.0, -800.0, 3.0]]), 5, 2.0,
                              ps.channel_centres(1.3e9, 1.31e9, 3), [5, 3])
    assert obs.K == 1
    src = ps.Source.centred(0.02, 0.01, 65, 2 * ps.ARCSEC)
    P = orc.patch_factored(obs, src)
    dobs = pk.DeviceObservation(obs)
    for prec in ACCURATE:
        err = orc.peak_normalised_error(gpu_patch(dobs, src, prec), P)[0]
        print(f"K=1 {prec}: {err:.3e}")
        assert err < TOL, (prec, err)


def test_ragged_bda_bins_and_long_k():
    obs = ps.tiny_random(32, n_ant=12, n_t=37, n_ch=7, nt=8, nc=3, radius_m=4000.0, bda=True)
    src = ps.Source.centred(-0.015, 0.02, 65, 1.5 * ps.ARCSEC)
    D = orc.decorr(obs, src.l0, src.m0)
    P = orc.patch_factored(obs, src, D)
    dobs = pk.DeviceObservation(obs)
    Dg = pk.decorr(dobs, src.l0, src.m0).cpu().numpy()
    assert np.max(np.abs(Dg - D)) < 2e-6
    for prec in ACCURATE:
        assert orc.peak_normalised_error(gpu_patch(dobs, src, prec), P)[0] < TOL


def test_single_sample_bins_and_phase_centre():
    obs = ps.tiny_random(33, n_ant=5, n_t=6, n_ch=2, nt=1, nc=1)
    dobs = pk.DeviceObservation(obs)
    Dg = pk.decorr(dobs, 0.03, -0.02).cpu().numpy()
    assert np.all(Dg == 1.0 + 0.0j)
    obs1 = ps.observation(1)
    D0 = pk.decorr(pk.DeviceObservation(obs1), 0.0, 0.0).cpu().numpy()
    assert np.all(D0 == 1.0 + 0.0j)



@pytest.mark.parametrize("nt,nc", [(6, 3), (3, 3)])
def test_waves_spanning_many_baselines(nt, nc):
    """One or two bins per baseline (78 baselines): every lane of a wave
    belongs to a different baseline than its neighbours, so each lane steps
    from the wave's bisection result to its own baseline."""
    obs = ps.tiny_random(35, n_ant=13, n_t=6, n_ch=3, nt=nt, nc=nc, radius_m=3000.0)
    assert obs.K == (6 // nt) * (3 // nc) * 78
    src = ps.Source.centred(0.011, -0.017, 33, 2 * ps.ARCSEC)
    D = orc.decorr(obs, src.l0, src.m0)
    dobs = pk.DeviceObservation(obs)
    Dg = pk.decorr(dobs, src.l0, src.m0).cpu().numpy()
    assert np.max(np.abs(Dg - D)) < 2e-6
    P = orc.patch_factored(obs, src, D)
    for prec in ACCURATE:
        assert orc.peak_normalised_error(gpu_patch(dobs, src, prec), P)[0] < TOL, prec


def test_small_row_steps():
    """Baselines of a few metres at a 0.05 arcsec cell: the 16-row step of
    every phase factor is 1e-4 to 1e-3 rad, where the split forms' row
    recurrence is least accurate per element (its rounded 2 cos t is
    ill-conditioned there), for every visibility at once."""
    obs = ps.tiny_random(51, n_ant=8, n_t=60, n_ch=4, nt=3, nc=2, radius_m=10.0, dt=60.0)
    src = ps.Source.centred(0.003, -0.002, 257, 0.05 * ps.ARCSEC)
    P = orc.patch_factored(obs, src)
    dobs = pk.DeviceObservation(obs)
    for prec in ACCURATE:
        err = orc.peak_normalised_error(gpu_patch(dobs, src, prec), P)[0]
        print(f"small row steps {prec}: {err:.2e}", flush=True)
        assert err < TOL, (prec, err)

def test_zero_weights_give_zero_patch():
    obs = ps.tiny_random(34, n_ant=4, n_t=9, n_ch=3, nt=3, nc=2)
    obs.W[:] = 0.0
    src = ps.Source.centred(0.01, 0.01, 33, 2 * ps.ARCSEC)
    dobs = pk.DeviceObservation(obs)
    for prec in ACCURATE:
        assert np.all(gpu_patch(dobs, src, prec) == 0.0)


def test_repeat_calls_bitwise_identical(cfg1):
    obs, dobs, src, D, P = cfg1
    a = gpu_patch(dobs, src, "split_bf16")
    b = gpu_patch(dobs, src, "split_bf16")
    assert np.array_equal(a, b)


@pytest.fixture(scope="module")
def cfg2():
    path = os.path.join(HERE, "golden", "config2_seed0_P.npy")
    if not os.path.exists(path):
        pytest.skip("config-2 golden patch not generated")
    obs = ps.observation(2, seed=0)
    src = ps.sources(2, seed=0)[0]
    return obs, pk.DeviceObservation(obs), src, np.load(path)


@pytest.mark.parametrize("prec", ACCURATE + ["mixed_fp16", "sr_fp16"])
def test_config2_full_patch(cfg2, prec):
    obs, dobs, src, P = cfg2
    Pg = gpu_patch(dobs, src, prec)
    err, rms = orc.peak_normalised_error(Pg, P)
    print(f"config2 {prec}: max {err:.3e} rms {rms:.3e}")
    assert err < TOL


def test_config2_decorr_sample(cfg2):
    obs, dobs, src, _ = cfg2
    smp = np.load(os.path.join(HERE, "golden", "config2_seed0_Dsample.npy"))
    ks = smp[:, 0].astype(np.int64)
    Dref = smp[:, 1] + 1j * smp[:, 2]
    Dg = pk.decorr(dobs, src.l0, src.m0).cpu().numpy()[ks]
    assert np.max(np.abs(Dg - Dref)) < 2e-6


def test_single_source_patch_graph_capture_and_replay(cfg1):
    """psf_patch (factors, contraction, finalise) captured in a HIP graph and
    replayed three times with unrelated eager work between replays: every
    replay equals the eager result bit for bit."""
    obs, dobs, src, _, P = cfg1
    ws = pk.Workspace()
    eager = pk.patch(dobs, src, prec="split_bf16", workspace=ws).clone()
    out = torch.zeros_like(eager)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pk.patch(dobs, src, prec="split_bf16", workspace=ws, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pk.patch(dobs, src, prec="split_bf16", workspace=ws, out=out)
    for rep in range(3):
        out.fill_(float("nan"))
        torch.randn(1 << 20, device="cuda").sum().item()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
    assert orc.peak_normalised_error(out.double().cpu().numpy(), P)[0] < TOL


def _empty_observation():
    """No baselines: K = 0 (every sum over visibilities is empty)."""
    return ps.Observation(ant_enu=np.zeros((2, 3)), bl_ant=np.zeros((0, 2), np.int32), times_s=np.zeros(4),
                          uvw_m=np.zeros((0, 4, 3)), freq_hz=np.array([1.4e9]), bl_bin=np.zeros((0, 2), np.int32),
                          bl_koff=np.zeros(1, np.int64), bl_tboff=np.zeros(1, np.int64), uvw_c_m=np.zeros((0, 3)),
                          W=np.zeros(0, np.float32))


def test_empty_observation_through_every_entry_point():
    """K = 0: the patch, the batched patches, the exact-w patch, the Method-2
    spectrum and patches and the adjoint are all zero, and CLEAN (host-driven
    and on the device) runs no cycle; the FP64 oracle's patch is zero too."""
    obs = _empty_observation()
    assert obs.K == 0
    src = ps.Source.centred(0.01, -0.02, 33, 2.0 * ps.ARCSEC)
    assert np.all(orc.patch_factored(obs, src) == 0.0)
    dobs = pk.DeviceObservation(obs)
    assert pk.decorr(dobs, src.l0, src.m0).numel() == 0
    for prec in ACCURATE:
        assert torch.count_nonzero(pk.patch(dobs, src, prec=prec)).item() == 0
    srcs = [src, ps.Source.centred(0.02, 0.0, 65, 2.0 * ps.ARCSEC)]
    assert torch.count_nonzero(pk.patch_batched(dobs, srcs)).item() == 0
    P, n = pk.patch_fullw(dobs, src)
    assert n == 1 and torch.count_nonzero(P).item() == 0
    S = pk.method2_spectrum(dobs, 64, src.dl)
    assert torch.count_nonzero(pk.method2_patches(S, src.dl, [(0.01, 0.0)], 20.0, 1e6, 1.4e9)).item() == 0
    G = torch.ones(sum(s.nl * s.nm for s in srcs), device="cuda")
    for prec in ("split_bf16", "fp32"):
        assert torch.count_nonzero(pk.patch_backward(dobs, srcs, G, prec)).item() == 0
    dirty = torch.ones((33, 33))
    res, comps = pk.clean_hogbom(dobs, src, dirty, 5)
    torch.cuda.synchronize()
    assert comps == [] and torch.equal(res.cpu(), dirty)
    res = dirty.to("cuda").clone()
    _, _, _, n_comp = pk.clean_hogbom_device(dobs, src, res, 5)
    torch.cuda.synchronize()
    assert int(n_comp.item()) == 0 and torch.equal(res.cpu(), dirty)


@pytest.mark.parametrize("prec", ACCURATE)
def test_normalised_patch(prec):
    """Row a6: P / (2 Re sum W D) from the library (PSF_NORMALISE) for a
    centred symmetric-size grid, a grid 300 pixels away from its source and
    a general-size grid, single and batched, against the oracle's normalised
    patch; an observation with every weight 0 gives zeros."""
    obs = ps.tiny_random(38, n_ant=10, n_t=25, n_ch=4, nt=5, nc=2, radius_m=3000.0)
    dobs = pk.DeviceObservation(obs)
    cell = 2 * ps.ARCSEC
    srcs = [ps.Source.centred(0.011, -0.007, 65, cell),
            _grid(-0.004, 0.016, 129, 129, cell, cell, shift_l=300.0, shift_m=-120.0),
            ps.Source.centred(0.02, 0.003, 40, cell, nm=50)]
    refs = [orc.patch_normalised(obs, s) for s in srcs]
    for s, ref in zip(srcs, refs):
        got = pk.patch(dobs, s, prec=prec, normalise=True)
        torch.cuda.synchronize()
        err = float(np.max(np.abs(got.double().cpu().numpy() - ref)))
        print(f"normalised {s.nl}x{s.nm} {prec}: {err:.2e}", flush=True)
        assert err < TOL * max(1.0, float(np.max(np.abs(ref))))
    parts = pk.split_patches(pk.patch_batched(dobs, srcs, prec=prec, normalise=True), srcs)
    torch.cuda.synchronize()
    for p, ref in zip(parts, refs):
        assert float(np.max(np.abs(p.double().cpu().numpy() - ref))) < TOL * max(1.0, float(np.max(np.abs(ref))))
    obs.W[:] = 0.0
    z = pk.patch(pk.DeviceObservation(obs), srcs[0], prec=prec, normalise=True)
    torch.cuda.synchronize()
    assert torch.count_nonzero(z).item() == 0


def test_normalise_flag_rejected_where_not_supported(cfg1):
    obs, dobs, src, _, _ = cfg1
    n = src.nl * src.nm
    with pytest.raises(pk.PsfError) as e:
        pk.patch_backward(dobs, [src], torch.zeros(n, device="cuda"), prec=pk.PSF_SPLIT_BF16 | pk.PSF_NORMALISE)
    assert e.value.status == pk.PSF_EINVAL
