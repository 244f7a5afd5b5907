"""The precision workload: 64 ants (2016 baselines), 1 h at 2 s, 64 channels
over 0.9-1.7 GHz averaged to 10 s x 2 channels (K = 23.2M visibilities), 64
sources at radii 0.1-3 deg with 257 x 257 patches at 1.5 arcsec, all in one
batched call per precision.  Split-BF16, split-FP16, mixed-FP16,
stochastic-FP16 and FP32 contractions against the FP64 oracle at sampled pixels of twelve sources,
from the nearest (0.2 deg) to the six farthest (2.94-2.96 deg) (max and
RMS, normalised by the patch's largest |P64|, <= 1e-5), and the split,
mixed and stochastic forms against the FP32 one over every pixel of all 64
PSFs (reported per PSF)."""
import json
import math
import os

import numpy as np
import pytest

import psf_synth as ps

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")
TOL = 1e-5


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2009_07010_amd as pk
    pk.lib()
    return pk


@pytest.fixture(scope="module")
def runs(pk):
    if not os.path.exists(os.path.join(GOLD, "config4_seed0_pixels.npy")):
        pytest.skip("golden values for workload 4 not generated")
    print("generating workload 4 (K = 23.2M)", flush=True)
    obs = ps.observation(4, seed=0)
    srcs = ps.sources(4, seed=0)
    dobs = pk.DeviceObservation(obs)
    out = {}
    for prec in ("fp32", "split_bf16", "split_fp16", "mixed_fp16", "sr_fp16"):
        P = pk.patch_batched(dobs, srcs, prec=prec)
        torch.cuda.synchronize()
        out[prec] = [p.double().cpu().numpy() for p in pk.split_patches(P, srcs)]
        print(f"workload 4 {prec}: 64 PSFs done", flush=True)
    return obs, srcs, out


def _scale(rows):
    """The error's normaliser, max |P64| over the patch, bounded below by what
    the golden rows hold: the largest stored |P64| and |P64(source)|.  Far
    sources of this wide band can have a small or negative P at the source
    itself (its bins decorrelate with either sign), so that value alone is
    not the patch's largest."""
    return max(abs(rows[0, 4]), float(np.max(np.abs(rows[:, 3]))))


def _gold():
    """Stored FP64 pixels of workload 4 from every golden file there is."""
    metas, rows = [], []
    for tag in ("config4_seed0", "config4_seed0_more"):
        if os.path.exists(os.path.join(GOLD, tag + "_pixels.npy")):
            metas.append(json.load(open(os.path.join(GOLD, tag + ".json"))))
            rows.append(np.load(os.path.join(GOLD, tag + "_pixels.npy")))
    return metas, np.concatenate(rows)


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16", "mixed_fp16", "sr_fp16", "fp32"])
def test_precision_workload_against_fp64(runs, prec):
    obs, srcs, out = runs
    metas, rows = _gold()
    assert all(obs.K == m["K"] for m in metas)
    for i in [i for m in metas for i in m["sources"]]:
        sel = rows[:, 0] == i
        ii, jj = rows[sel, 1].astype(int), rows[sel, 2].astype(int)
        d = (out[prec][i][ii, jj] - rows[sel, 3]) / _scale(rows[sel])
        emax, erms = np.max(np.abs(d)), math.sqrt(np.mean(d * d))
        r = math.degrees(math.hypot(srcs[i].l0, srcs[i].m0))
        print(f"workload 4 {prec} source {i} ({r:.2f} deg): max {emax:.2e} rms {erms:.2e}", flush=True)
        assert emax <= TOL


def test_precision_split_forms_against_fp32_every_pixel(runs):
    _, srcs, out = runs
    worst = 0.0
    print("src  r(deg)  bf16 max   bf16 rms   fp16 max   fp16 rms   mixed max  mixed rms  sr max     sr rms", flush=True)
    for i, s in enumerate(srcs):
        ref = out["fp32"][i]
        peak = np.max(np.abs(ref))
        line = f"{i:3d}  {math.degrees(math.hypot(s.l0, s.m0)):5.2f}"
        for prec in ("split_bf16", "split_fp16", "mixed_fp16", "sr_fp16"):
            d = (out[prec][i] - ref) / peak
            emax = float(np.max(np.abs(d)))
            worst = max(worst, emax)
            line += f"  {emax:.2e}  {math.sqrt(float(np.mean(d * d))):.2e}"
        print(line, flush=True)
    assert worst <= 2 * TOL
