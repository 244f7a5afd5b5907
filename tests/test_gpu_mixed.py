"""The FP16 contractions with stochastic rounding: the mixed form
(PSF_MIXED_FP16: the rows, cos and sin, as one stochastically rounded FP16
value each, the columns split hi + lo, two products) and the stochastic form
(PSF_SR_FP16: the columns too one stochastically rounded FP16 value, one
product); both run where the patch has the symmetric form and K >= 2^18.

Here, on a medium observation (30 antennas, 800 x 2 s, 64 channels over
1.3-1.5 GHz in 8 s x 2 channel bins, K = 2.78M): parity with the FP64
oracle at sampled pixels of the three symmetric families, on centred and
shifted grids and for a strongly decorrelated source (peak / sum |W D| =
0.17), <= 1e-5 of the patch's largest |P64| (bounded below by the sampled
pixels and the value at the source); bitwise repeatability; batched against
single calls; graph capture; and the routes to split-FP16 (small K,
patches without a symmetric form, the backward), which give split-FP16's
bits.  Its accuracy
on the full-size workloads is tested beside the other precisions (every
pixel of the uniform-bin 257 x 257 PSF, the precision workload's twelve
sources, the baseline-dependent workload's golden sources)."""
import numpy as np
import pytest

import oracle as orc
import psf_synth as ps

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = 1e-5
CELL = 1.5 * ps.ARCSEC
FORMS = ["mixed_fp16", "sr_fp16"]


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2009_07010_amd as pk
    pk.lib()
    return pk


@pytest.fixture(scope="module")
def medium(pk):
    obs = ps.tiny_random(7, n_ant=30, n_t=800, n_ch=64, nt=4, nc=2, radius_m=2000.0, dt=2.0)
    assert obs.K >= 1 << 18
    return obs, pk.DeviceObservation(obs)


def _source(r_deg, pa, n, shift=(0.0, 0.0), nm=None):
    l0, m0 = ps.direction(r_deg * ps.DEG, pa)
    nm = n if nm is None else nm
    return ps.Source(l0=l0, m0=m0, l_first=l0 - 0.5 * (n - 1) * CELL + shift[0] * CELL,
                     m_first=m0 - 0.5 * (nm - 1) * CELL + shift[1] * CELL, dl=CELL, dm=CELL, nl=n, nm=nm)


# (radius deg, position angle, rows, grid shift in pixels): the three
# symmetric families, centred and shifted grids, up to 2.5 deg
SOURCES = [(0.3, 0.7, 257, (0.0, 0.0)), (1.0, 2.1, 129, (0.0, 0.0)), (1.0, 4.0, 129, (0.37, -21.0)),
           (2.5, 5.2, 65, (0.0, 0.0)), (2.5, 1.3, 257, (-3.0, 40.0))]


def _pixels(n, g):
    """Centre, corners, edge midpoints, the centre's neighbours, and 24 random pixels."""
    c = n // 2
    ii = [c, 0, 0, n - 1, n - 1, c, c, 0, n - 1, c - 1, c + 1] + list(g.integers(0, n, 24))
    jj = [c, 0, n - 1, 0, n - 1, 0, n - 1, c, c, c, c] + list(g.integers(0, n, 24))
    return np.array(ii), np.array(jj)


@pytest.fixture(scope="module")
def refs(medium):
    obs, _ = medium
    g = np.random.default_rng(41)
    out = []
    for r, pa, n, sh in SOURCES:
        src = _source(r, pa, n, sh)
        D = orc.decorr(obs, src.l0, src.m0)
        ii, jj = _pixels(n, g)
        ref = orc.patch_pixels(obs, src, ii, jj, D=D)
        scale = max(float(np.max(np.abs(ref))), abs(2.0 * float(np.sum(obs.W * D).real)))
        out.append((src, ii, jj, ref, scale))
    return out


def test_against_oracle(pk, medium, refs):
    obs, dobs = medium
    for src, ii, jj, ref, scale in refs:
        P = {p: pk.patch(dobs, src, prec=p).double().cpu().numpy() for p in FORMS + ["split_fp16"]}
        err = {p: float(np.max(np.abs(v[ii, jj] - ref))) / scale for p, v in P.items()}
        r = np.degrees(np.hypot(src.l0, src.m0))
        print(f"{src.nl}^2 at {r:.1f} deg: " + " ".join(f"{p} {e:.2e}" for p, e in err.items()), flush=True)
        assert max(err.values()) <= TOL
        # the mixed and stochastic forms ran (their products differ from the split form's)
        assert np.any(P["mixed_fp16"] != P["split_fp16"]) and np.any(P["sr_fp16"] != P["mixed_fp16"])


@pytest.mark.parametrize("prec", FORMS)
def test_repeatable_and_batched(pk, medium, refs, prec):
    obs, dobs = medium
    srcs = [s for s, *_ in refs]
    a = pk.patch(dobs, srcs[0], prec=prec)
    b = pk.patch(dobs, srcs[0], prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    parts = pk.split_patches(pk.patch_batched(dobs, srcs, prec=prec), srcs)
    for (src, ii, jj, ref, scale), Pb in zip(refs, parts):
        Pb = Pb.double().cpu().numpy()
        Ps = pk.patch(dobs, src, prec=prec).double().cpu().numpy()
        # the same rounded operands (a bin's random word is its index), other
        # k-slices: the two differ by FP32 accumulation order only, which for
        # the strongly decorrelated source (sums of terms 6 times the patch's
        # peak) reaches 2e-6 of the peak over the whole patch
        d = float(np.max(np.abs(Pb - Ps))) / scale
        e = float(np.max(np.abs(Pb[ii, jj] - ref))) / scale
        print(f"{prec} batched {src.nl}^2: vs single {d:.2e}, vs FP64 {e:.2e}", flush=True)
        assert d <= TOL / 2 and e <= TOL


@pytest.mark.parametrize("prec", FORMS)
def test_routes_to_split_fp16(pk, medium, prec):
    obs, dobs = medium
    # a patch size without a symmetric form, K >= 2^18
    src = _source(1.0, 0.4, 100, nm=90)
    a = pk.patch(dobs, src, prec=prec)
    b = pk.patch(dobs, src, prec="split_fp16")
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # a symmetric-form patch with K < 2^18
    small = ps.tiny_random(3, n_ant=12, n_t=60, n_ch=8, nt=2, nc=2, radius_m=3000.0)
    assert small.K < 1 << 18
    ds = pk.DeviceObservation(small)
    src = _source(0.8, 1.0, 129)
    a = pk.patch(ds, src, prec=prec)
    b = pk.patch(ds, src, prec="split_fp16")
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    ref = orc.patch_factored(small, src)
    assert orc.peak_normalised_error(a.double().cpu().numpy(), ref)[0] <= TOL


@pytest.mark.parametrize("prec", FORMS)
def test_backward_takes_split_fp16(pk, medium, prec):
    obs, dobs = medium
    srcs = [_source(1.0, 2.1, 129), _source(2.5, 5.2, 65), _source(0.3, 0.7, 257)]
    g = torch.Generator(device="cpu").manual_seed(5)
    G = torch.randn(sum(s.nl * s.nm for s in srcs), generator=g, dtype=torch.float32)
    a = pk.patch_backward(dobs, srcs, G, prec)
    b = pk.patch_backward(dobs, srcs, G, "split_fp16")
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("prec", FORMS)
def test_graph_capture_and_replay_with_new_directions(pk, medium, refs, prec):
    """A batched call of the three symmetric families captured into a graph
    (after an eager call, which gives each kernel its registers' scratch):
    replays equal the eager result bit for bit, with unrelated eager work in
    between, and a replay after new directions are written to the device
    source array equals an eager call at those directions."""
    obs, dobs = medium
    srcs = [refs[0][0], refs[1][0], refs[3][0]]
    h, d = pk.device_sources(srcs)
    ws = pk.Workspace()
    total = sum(s.nl * s.nm for s in srcs)
    eager = pk.patch_batched(dobs, srcs, prec=prec, workspace=ws, d_srcs=d).clone()
    out = torch.zeros(total, dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream
        pk.patch_batched(dobs, srcs, prec=prec, workspace=ws, d_srcs=d, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pk.patch_batched(dobs, srcs, prec=prec, workspace=ws, d_srcs=d, out=out)
    for rep in range(3):
        out.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda")
        junk.sum().item()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
    moved = [s.with_direction(s.l0 + 2e-6, s.m0 - 3e-6) for s in srcs]
    pk.set_directions(d, torch.tensor([[s.l0, s.m0] for s in moved], dtype=torch.float64, device="cuda"))
    g.replay()
    torch.cuda.synchronize()
    eager2 = pk.patch_batched(dobs, moved, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(out, eager2)
    assert not torch.equal(eager2, eager)
