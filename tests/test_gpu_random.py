"""Seeded random parity cases: patch sizes of both forms (the general
form's tile families and the symmetric form's 65/129/257 rows with widths
across their families), grids centred on the source or many pixels off it,
cells of either sign and unequal along the axes, directions up to 3 deg,
uniform and baseline-dependent bins, every accurate precision, single and
batched calls, against the FP64 oracle's patch, peak-normalised (max |P64|
over the patch), <= 1e-5."""
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
            nl = int(g.choice([65, 129, 257]))
            nm = nl + int(g.integers(-15, 1)) if nl > 65 else nl - int(g.integers(0, 15))
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
