"""GPU parity of the batched path (psf_patch_batched: many sources and patch
sizes per call, persistent contraction, graph capture, autotuner) against
the FP64 oracle.  Bar: 1e-5 peak-normalised max error per patch."""
import json
import os
import time

import numpy as np
import pytest

import oracle as orc
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


def _mixed_sources():
    """Patch sizes of every compiled tile family (5, 9 and 17 blocks, the
    general 8-block tiling with ragged edges) at several directions."""
    cell = 1.5 * ps.ARCSEC
    spec = [(0.3, 40.0, 65, 65), (1.2, 200.0, 129, 129), (0.8, 300.0, 257, 257), (2.0, 10.0, 33, 16),
            (1.5, 120.0, 65, 65), (0.1, 250.0, 129, 129), (2.5, 80.0, 160, 161)]
    out = []
    for r, pa, nl, nm in spec:
        l0, m0 = ps.direction(r * ps.DEG, np.deg2rad(pa))
        out.append(ps.Source.centred(l0, m0, nl, cell, nm=nm))
    return out


def _err(P, ref):
    return orc.peak_normalised_error(np.asarray(P, np.float64), ref)[0]


@pytest.fixture(scope="module")
def bda_case():
    """A baseline-dependent-averaging observation with uneven bins (every
    baseline its own bin length in time and frequency)."""
    obs = ps.tiny_random(3, n_ant=12, n_t=120, n_ch=16, nt=12, nc=4, radius_m=4000.0, bda=True)
    return obs


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16"])
def test_batched_mixed_sizes_vs_oracle(pk, bda_case, prec):
    obs = bda_case
    srcs = _mixed_sources()
    dobs = pk.DeviceObservation(obs)
    P_all = pk.patch_batched(dobs, srcs, prec=prec)
    torch.cuda.synchronize()
    for s, P in zip(srcs, pk.split_patches(P_all, srcs)):
        ref = orc.patch_factored(obs, s)
        e = _err(P.cpu().numpy(), ref)
        print(f"batched {prec} {s.nl}x{s.nm}: {e:.2e}", flush=True)
        assert e <= TOL


def test_batched_agrees_with_single_source_calls(pk, bda_case):
    obs = bda_case
    srcs = _mixed_sources()
    dobs = pk.DeviceObservation(obs)
    P_all = pk.patch_batched(dobs, srcs, prec="split_bf16")
    for s, P in zip(srcs, pk.split_patches(P_all, srcs)):
        Q = pk.patch(dobs, s, prec="split_bf16")
        scale = torch.max(torch.abs(Q))
        assert torch.max(torch.abs(P - Q)) <= 2e-6 * scale


def test_batched_more_sources_than_one_group(pk):
    """More sources of one family than a launch takes (16), so several
    groups run back to back; repeated directions give equal patches."""
    obs = ps.observation(1)
    base = ps.sources(1)[0]
    srcs = []
    for n in range(37):
        l0, m0 = ps.direction((0.2 + 0.05 * (n % 9)) * ps.DEG, np.deg2rad(17.0 * n))
        srcs.append(ps.Source.centred(l0, m0, 65, 2.0 * ps.ARCSEC))
    srcs.append(base)
    srcs.append(base)
    dobs = pk.DeviceObservation(obs)
    parts = pk.split_patches(pk.patch_batched(dobs, srcs, prec="split_bf16"), srcs)
    torch.cuda.synchronize()
    for n in (0, 16, 36, 37):
        ref = orc.patch_factored(obs, srcs[n])
        assert _err(parts[n].cpu().numpy(), ref) <= TOL
    assert torch.equal(parts[-1], parts[-2])


def test_batched_graph_capture_and_replay_with_new_directions(pk, bda_case):
    obs = bda_case
    srcs = _mixed_sources()[:4]
    dobs = pk.DeviceObservation(obs)
    h, d = pk.device_sources(srcs)
    ws = pk.Workspace()
    total = sum(s.nl * s.nm for s in srcs)
    eager = pk.patch_batched(dobs, srcs, prec="split_bf16", workspace=ws, d_srcs=d).clone()
    out = torch.zeros(total, dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream
        pk.patch_batched(dobs, srcs, prec="split_bf16", workspace=ws, d_srcs=d, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pk.patch_batched(dobs, srcs, prec="split_bf16", workspace=ws, d_srcs=d, out=out)
    for rep in range(3):
        out.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda")  # unrelated eager work between replays
        junk.sum().item()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
    # new directions through the device source array, same grids
    moved = [s.with_direction(s.l0 + 2e-6, s.m0 - 3e-6) for s in srcs]
    pk.set_directions(d, torch.tensor([[s.l0, s.m0] for s in moved], dtype=torch.float64, device="cuda"))
    g.replay()
    torch.cuda.synchronize()
    eager2 = pk.patch_batched(dobs, moved, prec="split_bf16", workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(out, eager2)
    for s, P in zip(moved, pk.split_patches(out, moved)):
        assert _err(P.cpu().numpy(), orc.patch_factored(obs, s)) <= TOL


def test_autotune_table_drives_batched_launch(pk, bda_case):
    obs = bda_case
    srcs = _mixed_sources()
    dobs = pk.DeviceObservation(obs)
    table = pk.autotune(dobs, srcs, prec="split_bf16")
    doc = json.loads(table)
    fams = {(f["tbi0"], f["tbi1"], f["tbj0"], f["tbj1"], f["sym"]) for f in doc["families"]}
    # symmetric form for the 65-, 129- and 257-row patches, the general
    # form's 8 x 8 tiles else
    assert fams == {(5, 5, 5, 5, 1), (9, 9, 9, 9, 1), (9, 8, 17, 17, 1), (8, 8, 8, 8, 0)}
    for f in doc["families"]:
        assert 1 <= f["items_per_cu"] <= 4 and f["flush"] in (32, 64, 128) and f["ms"] > 0
    P_all = pk.patch_batched(dobs, srcs, prec="split_bf16", tuning=table)
    torch.cuda.synchronize()
    for s, P in zip(srcs, pk.split_patches(P_all, srcs)):
        assert _err(P.cpu().numpy(), orc.patch_factored(obs, s)) <= TOL


def test_batched_rejects_bad_tuning_table(pk, bda_case):
    dobs = pk.DeviceObservation(bda_case)
    srcs = _mixed_sources()[:1]
    bad = '{"families": [{"tbi0": 5, "tbi1": 5, "tbj0": 5, "tbj1": 5, "items_per_cu": 99, "flush": 64}]}'
    with pytest.raises(pk.PsfError) as e:
        pk.patch_batched(dobs, srcs, tuning=bad)
    assert e.value.status == pk.PSF_EINVAL


@pytest.fixture(scope="module")
def config5():
    if not os.path.exists(os.path.join(GOLD, "config5_seed0_pixels.npy")):
        pytest.skip("golden values for workload 5 not generated")
    print("generating workload 5 (K ~ 2.65e8)", flush=True)
    return ps.observation(5, seed=0)


@pytest.mark.parametrize("prec", ["split_bf16", "mixed_fp16", "sr_fp16", "fp32"])
def test_batched_config5_sampled_pixels(pk, config5, prec):
    """Workload 5 at full size (baseline-dependent averaging, K ~ 2.65e8):
    the golden sources (one per patch size) batched with 9 more, compared
    with the FP64 oracle at sampled pixels, normalised by the patch peak
    2 Re sum W D."""
    obs = config5
    meta = json.load(open(os.path.join(GOLD, "config5_seed0.json")))
    assert obs.K == meta["K"]
    rows = np.load(os.path.join(GOLD, "config5_seed0_pixels.npy"))
    all_srcs = ps.sources(5, seed=0)
    idx = list(meta["sources"]) + [i for i in range(12) if i not in meta["sources"]][:9]
    srcs = [all_srcs[i] for i in idx]
    dobs = pk.DeviceObservation(obs)
    parts = pk.split_patches(pk.patch_batched(dobs, srcs, prec=prec), srcs)
    torch.cuda.synchronize()
    for q, i in enumerate(meta["sources"]):
        sel = rows[:, 0] == i
        ii, jj = rows[sel, 1].astype(int), rows[sel, 2].astype(int)
        ref, peak = rows[sel, 3], max(abs(rows[sel, 4][0]), float(np.max(np.abs(rows[sel, 3]))))
        got = parts[q].cpu().numpy().astype(np.float64)[ii, jj]
        e = np.max(np.abs(got - ref)) / abs(peak)
        print(f"config5 {prec} source {i} ({srcs[q].nl}^2): {e:.2e}", flush=True)
        assert e <= TOL


def _config5_gold():
    """Stored FP64 pixels of workload 5: {source index: (i, j, P_ij, scale)},
    scale the error's normaliser (max |P64| over the patch, bounded below by
    the stored pixels and the value at the source)."""
    out = {}
    for name in ("config5_seed0_pixels.npy", "config5_seed0_far_pixels.npy"):
        f = os.path.join(GOLD, name)
        if not os.path.exists(f):
            continue
        rows = np.load(f)
        for i in np.unique(rows[:, 0]).astype(int):
            sel = rows[:, 0] == i
            # normaliser: max |P64| over the patch, bounded below by the stored pixels and the source's value
            out[int(i)] = (rows[sel, 1].astype(int), rows[sel, 2].astype(int), rows[sel, 3],
                           max(abs(rows[sel, 4][0]), float(np.max(np.abs(rows[sel, 3])))))
    return out


def test_batched_config5_all_256_sources_one_graph(pk, config5):
    """Workload 5 at full size, every one of its 256 sources (65, 129 and
    257 pixels a side, 0.05-3 deg) in one psf_patch_batched call captured
    into a HIP graph; the replay's patches of every source with stored FP64
    pixels (the first of each size, and the largest radius of each size)
    against the oracle, peak-normalised."""
    obs = config5
    srcs = ps.sources(5, seed=0)
    assert len(srcs) == 256
    gold = _config5_gold()
    dobs = pk.DeviceObservation(obs)
    ws = pk.Workspace()
    ws.get(pk.workspace_bytes(dobs, srcs, "split_bf16"))
    _, d = pk.device_sources(srcs)
    out = torch.full((sum(s.nl * s.nm for s in srcs),), float("nan"), dtype=torch.float32, device="cuda")
    first = [next(s for s in srcs if s.nl == n) for n in (65, 129, 257)]
    pk.patch_batched(dobs, first, workspace=ws)  # every tile family's kernels loaded outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pk.patch_batched(dobs, srcs, out=out, workspace=ws, d_srcs=d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    terms = float(obs.K) * sum(s.nl * s.nm for s in srcs)
    print(f"workload 5, 256 sources in one graph replay: {wall:.2f} s, {terms / wall:.3e} terms/s", flush=True)
    assert torch.isfinite(out).all()
    parts = pk.split_patches(out, srcs)
    assert len(gold) >= 3
    for i, (ii, jj, ref, peak) in sorted(gold.items()):
        got = parts[i].cpu().numpy().astype(np.float64)[ii, jj]
        e = np.max(np.abs(got - ref)) / abs(peak)
        r = np.degrees(np.arcsin(np.hypot(srcs[i].l0, srcs[i].m0)))
        print(f"workload 5 source {i} ({srcs[i].nl}^2 at {r:.2f} deg): {e:.2e}", flush=True)
        assert e <= TOL
