"""psf_patch_noalloc (the entry point that allocates nothing, on the
library's fixed scratch) against psf_patch with a workspace: bit-identical
patches on two calls in a row, the second with a smaller observation and
patch, and a clean PSF_EWORKSPACE where the fixed scratch is too small."""
import numpy as np
import pytest

import oracle as orc
import psf_synth as ps

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2009_07010_amd as pk
    pk.lib()
    return pk


@pytest.mark.parametrize("prec", ["split_bf16", "fp32"])
def test_noalloc_matches_workspace_call(pk, prec):
    big_obs, big_src = ps.observation(2), ps.sources(2)[0]            # K = 5.8M, 257 x 257
    small_obs, small_src = ps.observation(1), ps.sources(1)[0]        # K = 420, 65 x 65
    ragged = ps.Source.centred(small_src.l0, small_src.m0, 40, 2 * ps.ARCSEC, nm=50)
    cases = [(pk.DeviceObservation(big_obs), big_src, False), (pk.DeviceObservation(small_obs), small_src, False),
             (pk.DeviceObservation(small_obs), ragged, True)]
    for dobs, src, norm in cases:
        got = pk.patch_noalloc(dobs, src, prec=prec, normalise=norm)
        ref = pk.patch(dobs, src, prec=prec, normalise=norm)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        print(f"noalloc K={dobs.K} {src.nl}x{src.nm} {prec} normalise={norm}: "
              f"max |diff| {np.max(np.abs(g - r)):.2e}", flush=True)
        assert np.array_equal(g, r)
    # the small patch against the FP64 oracle as well
    P = orc.patch_factored(small_obs, small_src)
    err = orc.peak_normalised_error(pk.patch_noalloc(cases[1][0], small_src, prec=prec).double().cpu().numpy(), P)[0]
    assert err < 1e-5


def test_noalloc_rejects_what_does_not_fit(pk):
    obs = ps.observation(4)   # K = 23.2M: 930 MB of records alone
    src = ps.sources(4)[0]
    with pytest.raises(pk.PsfError) as e:
        pk.patch_noalloc(pk.DeviceObservation(obs), src)
    assert e.value.status == pk.PSF_EWORKSPACE and "scratch" in str(e.value)
