"""GPU parity of Hogbom CLEAN with position-dependent PSFs (psf_clean_hogbom,
the paper's Algorithm 2) against the FP64 oracle on the same dirty image.
Components: identical pixels, amplitudes within 1e-5 of the dirty peak;
residual within 1e-5 of the dirty peak.  The device-resident variant
(psf_clean_hogbom_device) equals the host-driven one bit for bit, eagerly
and replayed from a captured graph."""
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


def _setup(sources, n=65):
    obs = ps.observation(1)
    grid = ps.Source.centred(0.004, -0.003, n, 2.0 * ps.ARCSEC)
    dirty = sum(f * orc.patch_factored(obs, grid.with_direction(grid.l_first + i * grid.dl,
                                                                grid.m_first + j * grid.dm))
                for i, j, f in sources)
    return obs, grid, dirty


def _compare(pk, obs, grid, dirty, gain, n_iter, prec, threshold=0.0):
    ref_res, ref_comps = orc.hogbom_clean(obs, grid, dirty, gain, n_iter, threshold)
    dobs = pk.DeviceObservation(obs)
    res, comps = pk.clean_hogbom(dobs, grid, torch.as_tensor(dirty, dtype=torch.float32), n_iter, gain, threshold,
                                 prec=prec)
    scale = np.max(np.abs(dirty))
    assert [c[:2] for c in comps] == [c[:2] for c in ref_comps]
    amp_err = max([abs(a - b[2]) for (_, _, a), b in zip(comps, ref_comps)] + [0.0]) / scale
    res_err = np.max(np.abs(res.double().cpu().numpy() - ref_res)) / scale
    print(f"{prec}: {len(comps)} components, amplitude err {amp_err:.2e}, residual err {res_err:.2e}", flush=True)
    assert amp_err <= TOL and res_err <= TOL
    return ref_res, ref_comps


@pytest.mark.parametrize("prec", ["split_bf16", "fp32"])
def test_clean_single_source_geometric(pk, prec):
    obs, grid, dirty = _setup([(20, 11, 0.7)])
    ref_res, comps = _compare(pk, obs, grid, dirty, 0.3, 6, prec)
    assert all(c[:2] == (20, 11) for c in comps)


@pytest.mark.parametrize("prec", ["split_bf16", "fp32"])
def test_clean_three_sources_matches_oracle(pk, prec):
    obs, grid, dirty = _setup([(10, 12, 1.0), (50, 44, 0.45), (33, 52, 0.2)])
    _compare(pk, obs, grid, dirty, 0.5, 10, prec)


def test_clean_threshold_stops_before_any_cycle(pk):
    obs, grid, dirty = _setup([(20, 11, 0.7)], n=33)
    dobs = pk.DeviceObservation(obs)
    d = torch.as_tensor(dirty, dtype=torch.float32)
    res, comps = pk.clean_hogbom(dobs, grid, d, 5, 0.2, float(np.max(np.abs(dirty))) * 1.01)
    assert comps == [] and torch.equal(res.cpu(), d)


@pytest.mark.parametrize("N", [128, 32])
def test_clean_with_method2_psfs_matches_oracle(pk, N):
    """CLEAN with the Method-2 PSF at every peak (N = 128 covers the 65-pixel
    image from any peak; N = 32 is cut, so pixels beyond its extent stay)."""
    obs, grid, dirty = _setup([(10, 12, 1.0), (50, 44, 0.45), (33, 52, 0.2)])
    dt, dnu, nu = 30.0, 1e6, 1.4e9
    Peff = orc.method2_effective_psf(obs, N, grid.dl)
    ref_res, ref_comps = orc.hogbom_clean_method2(Peff, grid, dirty, 0.5, 10, dt, dnu, nu)
    S = pk.method2_spectrum(pk.DeviceObservation(obs), N, grid.dl)
    res, comps = pk.clean_hogbom_method2(S, grid, torch.as_tensor(dirty, dtype=torch.float32), 10, dt, dnu, nu,
                                         gain=0.5)
    scale = np.max(np.abs(dirty))
    assert [c[:2] for c in comps] == [c[:2] for c in ref_comps]
    amp_err = max(abs(a - b[2]) for (_, _, a), b in zip(comps, ref_comps)) / scale
    res_err = np.max(np.abs(res.double().cpu().numpy() - ref_res)) / scale
    print(f"method-2 CLEAN N={N}: {len(comps)} components, amplitude err {amp_err:.2e}, residual err {res_err:.2e}",
          flush=True)
    assert amp_err <= TOL and res_err <= TOL


@pytest.mark.parametrize("prec", ["split_bf16", "fp32"])
def test_clean_on_device_equals_host_clean_and_oracle(pk, prec):
    """psf_clean_hogbom_device (peak placed on the device, a fixed number of
    cycles) against psf_clean_hogbom on the same dirty image, with a
    threshold that stops the cleaning after a few cycles: the same
    components and the same residual bit for bit, the cycles past the
    threshold subtracting nothing; and against the oracle."""
    obs, grid, dirty = _setup([(10, 12, 1.0), (50, 44, 0.45), (33, 52, 0.2)])
    gain, n_iter = 0.5, 12
    thr = 0.1 * float(np.max(np.abs(dirty)))  # reached after 8 cycles (the residual peak then 0.083 of it)
    ref_res, ref_comps = orc.hogbom_clean(obs, grid, dirty, gain, n_iter, thr)
    dobs = pk.DeviceObservation(obs)
    d = torch.as_tensor(dirty, dtype=torch.float32)
    host_res, host_comps = pk.clean_hogbom(dobs, grid, d, n_iter, gain, thr, prec=prec)
    assert 0 < len(host_comps) < n_iter
    res = d.to("cuda").clone()
    ci, cj, ca, n = pk.clean_hogbom_device(dobs, grid, res, n_iter, gain, thr, prec=prec)
    torch.cuda.synchronize()
    k = int(n.item())
    comps = [(int(a), int(b), float(c)) for a, b, c in zip(ci[:k].cpu(), cj[:k].cpu(), ca[:k].cpu())]
    print(f"device CLEAN {prec}: {k} components in {n_iter} cycles", flush=True)
    assert comps == host_comps
    assert torch.equal(res, host_res)
    assert [c[:2] for c in comps] == [c[:2] for c in ref_comps]
    scale = np.max(np.abs(dirty))
    assert np.max(np.abs(res.double().cpu().numpy() - ref_res)) / scale <= TOL


def test_clean_on_device_graph_replay(pk):
    """The device CLEAN captured once into a HIP graph and replayed three
    times, the residual reset to the dirty image (eager copies) and unrelated
    eager work between replays: every replay equals the eager call bit for
    bit, components included."""
    obs, grid, dirty = _setup([(10, 12, 1.0), (50, 44, 0.45)])
    dobs = pk.DeviceObservation(obs)
    ws = pk.Workspace()
    d = torch.as_tensor(dirty, dtype=torch.float32, device="cuda")
    res = d.clone()
    comps = pk.clean_hogbom_device(dobs, grid, res, 6, 0.4, 0.0, workspace=ws)
    torch.cuda.synchronize()
    eager = (res.clone(), *[c.clone() for c in comps])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        res.copy_(d)
        pk.clean_hogbom_device(dobs, grid, res, 6, 0.4, 0.0, workspace=ws, comps=comps)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pk.clean_hogbom_device(dobs, grid, res, 6, 0.4, 0.0, workspace=ws, comps=comps)
    for r in range(3):
        res.copy_(d)
        for c in comps:
            c.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(res, eager[0]), f"replay {r}: residual"
        for a, b in zip(comps, eager[1:]):
            assert torch.equal(a, b), f"replay {r}: components"
        _ = torch.randn(1024, device="cuda").sum()  # unrelated eager work between replays


def test_clean_on_device_zero_cycles_and_threshold_above_peak(pk):
    """No cycle asked for, and a threshold above the dirty peak: the residual
    is the dirty image and no component is recorded (the count is written
    by the call itself, whatever the arrays held)."""
    obs, grid, dirty = _setup([(20, 11, 0.7)], n=33)
    dobs = pk.DeviceObservation(obs)
    d = torch.as_tensor(dirty, dtype=torch.float32, device="cuda")
    for n_iter, thr in ((0, 0.0), (4, float(np.max(np.abs(dirty))) * 1.01)):
        res = d.clone()
        comps = [torch.full((max(1, n_iter),), -3, dtype=torch.int32, device="cuda"),
                 torch.full((max(1, n_iter),), -3, dtype=torch.int32, device="cuda"),
                 torch.zeros(max(1, n_iter), dtype=torch.float32, device="cuda"),
                 torch.full((1,), 99, dtype=torch.int32, device="cuda")]
        pk.clean_hogbom_device(dobs, grid, res, n_iter, 0.2, thr, comps=comps)
        torch.cuda.synchronize()
        assert int(comps[3].item()) == 0 and torch.equal(res, d)


@pytest.mark.parametrize("N", [128, 32])
def test_clean_method2_on_device_equals_host_clean(pk, N):
    """psf_clean_hogbom_method2_device against psf_clean_hogbom_method2 (a
    threshold that stops it part way at N = 128; N = 32 lays a cut PSF): the same
    components and residual bit for bit; then the device loop captured once
    and replayed twice from the dirty image, each replay equal again."""
    obs, grid, dirty = _setup([(10, 12, 1.0), (50, 44, 0.45), (33, 52, 0.2)])
    dt, dnu, nu, gain, n_iter = 30.0, 1e6, 1.4e9, 0.5, 12
    thr = 0.1 * float(np.max(np.abs(dirty)))
    S = pk.method2_spectrum(pk.DeviceObservation(obs), N, grid.dl)
    d = torch.as_tensor(dirty, dtype=torch.float32, device="cuda")
    host_res, host_comps = pk.clean_hogbom_method2(S, grid, d, n_iter, dt, dnu, nu, gain=gain, threshold=thr)
    # N = 128 stops at the threshold after 8 cycles; the cut N = 32 PSF leaves
    # sidelobes above it, so there every cycle subtracts
    assert 0 < len(host_comps) <= n_iter and (N != 128 or len(host_comps) < n_iter)
    ws = pk.Workspace()
    res = d.clone()
    comps = pk.clean_hogbom_method2_device(S, grid, res, n_iter, dt, dnu, nu, gain=gain, threshold=thr, workspace=ws)
    torch.cuda.synchronize()
    k = int(comps[3].item())
    got = [(int(a), int(b), float(c)) for a, b, c in zip(comps[0][:k].cpu(), comps[1][:k].cpu(), comps[2][:k].cpu())]
    print(f"device method-2 CLEAN N={N}: {k} components in {n_iter} cycles", flush=True)
    assert got == host_comps and torch.equal(res, host_res)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pk.clean_hogbom_method2_device(S, grid, res, n_iter, dt, dnu, nu, gain=gain, threshold=thr, workspace=ws,
                                       comps=comps)
    for r in range(2):
        res.copy_(d)
        comps[3].fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(res, host_res) and int(comps[3].item()) == k, f"replay {r}"
