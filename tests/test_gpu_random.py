"""Seeded random parity cases: patch sizes of both forms (the general
form's tile families and the symmetric form's 65/129/257 rows with widths
across their families), grids centred on the source or many pixels off it,
cells of either sign and unequal along the axes, directions up to 3 deg,
uniform and baseline-dependent bins, every accurate precision, single and
batched calls, against the FP64 oracle's patch, peak-normalised (max |P64|
over the patch), <= 1e-5; and the mixed and stochastic FP16 forms on random
observations large enough for them to run, at sampled pixels."""
import numpy as np
import pytest

import oracle as orc
import psf_synth as ps

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = 1e-5
ACCURATE = ("split_bf16", "split_fp16", "fp32")


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2009_07010_amd as pk
    pk.lib()
    return pk


def _case(seed):
    """One random (observation, sources, precision) case from its seed."""
    g = np.random.default_rng(9000 + seed)
    obs = ps.tiny_random(200 + seed, n_ant=int(g.integers(6, 12)), n_t=int(g.integers(20, 60)),
                         n_ch=int(g.integers(2, 9)), nt=int(g.integers(1, 6)), nc=int(g.integers(1, 4)),
                         radius_m=float(g.uniform(1000.0, 6000.0)), bda=bool(g.integers(0, 2)))
    srcs = []
    for _ in range(int(g.integers(1, 4))):
        r = g.uniform(0.0, 3.0) * ps.DEG
        l0, m0 = ps.direction(r, g.uniform(0.0, 2.0 * np.pi))
        if g.integers(0, 2):
            # a symmetric family: nm within the family's column blocks
            nl = int(g.choice([65, 129, 257]))
            nm = nl + int(g.integers(0, 16))
        else:
            nl, nm = int(g.integers(1, 300)), int(g.integers(1, 300))
        cell = g.uniform(0.5, 3.0) * ps.ARCSEC
        dl = cell * (1 if g.integers(0, 2) else -1)
        dm = cell * g.uniform(0.7, 1.4)
        sl = float(g.choice([0.0, g.uniform(-80.0, 80.0)]))
        sm = float(g.choice([0.0, g.uniform(-80.0, 80.0)]))
        srcs.append(ps.Source(l0=l0, m0=m0, l_first=l0 - 0.5 * (nl - 1) * dl + sl * dl,
                              m_first=m0 - 0.5 * (nm - 1) * dm + sm * dm, dl=dl, dm=dm, nl=nl, nm=nm))
    prec = ACCURATE[int(g.integers(0, 3))]
    return obs, srcs, prec


@pytest.mark.parametrize("seed", range(16))
def test_random_case_single_and_batched(pk, seed):
    obs, srcs, prec = _case(seed)
    dobs = pk.DeviceObservation(obs)
    refs = [orc.patch_factored(obs, s) for s in srcs]
    batched = pk.split_patches(pk.patch_batched(dobs, srcs, prec=prec), srcs)
    for s, ref, Pb in zip(srcs, refs, batched):
        P = pk.patch(dobs, s, prec=prec)
        torch.cuda.synchronize()
        e1 = orc.peak_normalised_error(P.double().cpu().numpy(), ref)[0]
        e2 = orc.peak_normalised_error(Pb.double().cpu().numpy(), ref)[0]
        print(f"seed {seed} K={obs.K} {s.nl}x{s.nm} {prec}: single {e1:.2e} batched {e2:.2e}", flush=True)
        assert e1 <= TOL and e2 <= TOL


def _medium_case(seed):
    """A random observation with K >= 2^18 bins (so that the mixed and
    stochastic forms run), one source of a symmetric family whose peak is
    at least 0.2 of sum |W D| (drawn again otherwise: the forms' error
    bound is stated relative to sum |W D|, so a nearly cancelled peak is
    outside what these cases check), sampled pixels, and D from the oracle."""
    g = np.random.default_rng(7000 + seed)
    while True:
        obs = ps.tiny_random(300 + int(g.integers(0, 1 << 20)), n_ant=int(g.integers(24, 33)),
                             n_t=int(g.integers(600, 801)), n_ch=int(g.integers(16, 33)), nt=int(g.integers(2, 7)),
                             nc=int(g.integers(1, 3)), radius_m=float(g.uniform(1000.0, 3000.0)),
                             dt=float(g.uniform(1.0, 3.0)), bda=bool(g.integers(0, 2)))
        r = g.uniform(0.05, 3.0) * ps.DEG
        l0, m0 = ps.direction(r, g.uniform(0.0, 2.0 * np.pi))
        if obs.K < 1 << 18:
            continue
        D = orc.decorr(obs, l0, m0)
        c = obs.W * D
        if np.sum(c.real) >= 0.2 * np.sum(np.abs(c)):
            break
    nl = (65, 129, 257)[seed % 3]  # every family twice over the six seeds
    nm = nl + int(g.integers(0, 16))  # within the family's column blocks
    cell = g.uniform(0.5, 3.0) * ps.ARCSEC
    dl = cell * (1 if g.integers(0, 2) else -1)
    dm = cell * g.uniform(0.7, 1.4)
    sl = float(g.choice([0.0, g.uniform(-40.0, 40.0)]))
    sm = float(g.choice([0.0, g.uniform(-40.0, 40.0)]))
    src = ps.Source(l0=l0, m0=m0, l_first=l0 - 0.5 * (nl - 1) * dl + sl * dl,
                    m_first=m0 - 0.5 * (nm - 1) * dm + sm * dm, dl=dl, dm=dm, nl=nl, nm=nm)
    h = (nl // 2, nm // 2)
    ii = np.array([h[0], 0, nl - 1, h[0], h[0], h[0] - 1, h[0] + 1] + list(g.integers(0, nl, 20)))
    jj = np.array([h[1], h[1], h[1], 0, nm - 1, h[1], h[1]] + list(g.integers(0, nm, 20)))
    return obs, src, ii, jj, D


@pytest.mark.parametrize("seed", range(6))
def test_random_stochastic_forms(pk, seed):
    """The mixed and stochastic FP16 forms on random observations of 2^18 to
    a few million bins (uniform or baseline-dependent bins) and random
    symmetric-family grids, against the FP64 oracle at 27 sampled pixels,
    normalised by the largest |P64| there and at the source (a lower bound
    of the patch's peak)."""
    obs, src, ii, jj, D = _medium_case(seed)
    assert obs.K >= 1 << 18
    ref = orc.patch_pixels(obs, src, ii, jj, D=D)
    scale = max(float(np.max(np.abs(ref))), abs(2.0 * float(np.sum(obs.W * D).real)))
    dobs = pk.DeviceObservation(obs)
    split = pk.patch(dobs, src, prec="split_fp16").cpu().numpy()
    for prec in ("mixed_fp16", "sr_fp16"):
        P = pk.patch(dobs, src, prec=prec).double().cpu().numpy()
        assert not np.array_equal(P, split)  # its own kernel ran, not the split-FP16 route
        e = float(np.max(np.abs(P[ii, jj] - ref))) / scale
        r = np.degrees(np.hypot(src.l0, src.m0))
        print(f"seed {seed} K={obs.K} {src.nl}x{src.nm} at {r:.2f} deg {prec}: {e:.2e}", flush=True)
        assert e <= TOL
