"""Throughput of the distorted-PSF hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec sr_fp16]

Headline workload: baseline-dependent averaging of a MeerKAT-shaped array
(64 antennas, 2016 baselines, 14400 x 1 s, 64 channels over 1.3-1.5 GHz,
per-baseline bins of floor(B_max/|b|) clamped to 1-64 samples x 1-8
channels: K = 265,127,960 averaged visibilities) with 256 sources at
0.05-3 deg whose patches are 65, 129 or 257 pixels square at 1.5".  One
step = one replay of a captured HIP graph holding one psf_patch_batched
call over 16 of the sources (decorrelation, phase factors, contraction
and finalise of each); steps cycle through the 16 slices, so 16 steps
cover all 256 sources.  The value is vis.pixel terms/s (K x nl x nm
one-sided terms per PSF) over the timed steps, in the stochastic FP16
arithmetic (rows and columns one stochastically rounded FP16 value each:
one matrix-core product per term product), whose error against the FP64
oracle at the stored pixels is part of the line.

Also printed, as keyed sub-entries: the headline in split-BF16 (three
products); one PSF of the uniform-bin workload (K = 5.8M, 257^2) in the
headline arithmetic, split-BF16 and plain FP32; the precision workload
(K = 23.2M, 64 sources of 257^2) in split-BF16, split-FP16, mixed-FP16
(rows stochastically rounded, columns split: two products), stochastic-FP16
and FP32; the
roofline of the contraction kernel from HIP events on its launch stream;
the paper's two approximations, CLEAN, windows, exact w, the adjoint; and
the FP64 CPU reference timed on a bounded sample of the headline workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"split_bf16": 2516.6, "split_fp16": 2516.6, "mixed_fp16": 2516.6, "sr_fp16": 2516.6,
               "plain_bf16": 2516.6, "fp32": 157.3}
# algorithmic work per useful one-sided term: 2 real multiply-adds
# (Re c a Re b - Im c a Im b), 4 flops, whatever the arithmetic
ALG_FLOPS_PER_TERM = 4.0
# matrix-core products per term product: 3 for the split forms (hi hi, hi lo, lo hi),
# 2 for the mixed form (rows once, columns hi and lo), 1 for the stochastic form
# (the last two for the symmetric form and K >= 2^18, else they run split-FP16)
PRODUCTS = {"split_bf16": 3, "split_fp16": 3, "mixed_fp16": 2, "sr_fp16": 1, "plain_bf16": 1, "fp32": 1}
MIXED_MIN_K = 1 << 18
DTYPE = {"split_bf16": "bf16", "split_fp16": "fp16", "mixed_fp16": "fp16", "sr_fp16": "fp16", "plain_bf16": "bf16",
         "fp32": "f32"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prec", default="sr_fp16", choices=list(PEAK_TFLOPS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baselines", type=int, default=72,
                    help="baselines of the headline workload in the CPU-reference sample")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="if > 0: only run this many headline steps of --prec (for rocprofv3) and print "
                         "nothing else")
    ap.add_argument("--profile-workload", default="bda256",
                    choices=["bda256", "meerkat257", "forward129", "adjoint129", "decorr-bda", "decorr-meerkat"],
                    help="what --profile-steps runs: headline graph replays, single uniform-bin PSFs, the "
                         "16-source 129x129 forward or adjoint, or decorrelation factors of one source "
                         "(headline or uniform-bin workload)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="if > 0: only copy a buffer of this many MiB a few times (calibrates the HBM "
                         "byte counters against a plain copy kernel) and print nothing else")
    return ap.parse_args()


KERNEL_SRC = os.path.join(ROOT, "paper_2009_07010_amd", "csrc", "k_patch.hip")


def measured_traffic(prec, workload="meerkat257"):
    """HBM bytes per contraction launch from the committed counter summary
    of this workload and precision, or None when there is none or the kernel
    source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_patch_traffic_{workload}_{prec}.txt")
    try:
        kv = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        with open(KERNEL_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        if kv.get("source_sha256") != sha or kv.get("precision") != prec:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def time_prec(pk, torch, dobs, src, prec, steps, warmup, ws):
    for _ in range(warmup):
        pk.patch(dobs, src, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    out = torch.empty((src.nl, src.nm), dtype=torch.float32, device="cuda")
    pk.psf_timing_read()
    pk.psf_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pk.patch(dobs, src, prec=prec, workspace=ws, out=out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, nk = pk.psf_timing_read()
    pk.psf_timing_enable(False)
    return wall / steps * 1e3, kms / max(nk, 1), out


def time_method1(pk, torch, dobs, src, prec, ws, reps=10):
    """The paper's Method 1 on the same workload: its closed-form (sinc)
    decorrelation factors against the exact ones (reads only each bin's end
    rows, about 80 bytes per bin), and the PSF built from them."""
    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    D = torch.empty((dobs.K, 2), dtype=torch.float32, device="cuda")
    sinc_ms = timed(lambda: pk.decorr_sinc(dobs, src.l0, src.m0, out=D))
    exact_ms = timed(lambda: pk.decorr(dobs, src.l0, src.m0, out=D))
    Dc = pk.decorr_sinc(dobs, src.l0, src.m0)
    psf_ms = timed(lambda: pk.patch(dobs, src, prec=prec, D=Dc, workspace=ws))
    # exact factors: every uvw row (24 B), every time-bin centre (24 B) and
    # D (8 B per bin) once; every sample's phase is evaluated
    exact_bytes = 24.0 * dobs.n_bl * dobs.n_t + 24.0 * dobs.n_tb + 8.0 * dobs.K
    samples = float(dobs.n_bl) * dobs.n_t * dobs.n_ch
    return {"decorr_sinc_ms": sinc_ms, "decorr_exact_ms": exact_ms,
            "decorr_sinc_GBps": 80.0 * dobs.K / (sinc_ms * 1e-3) / 1e9,
            "decorr_exact_GBps": exact_bytes / (exact_ms * 1e-3) / 1e9,
            "decorr_exact_hbm_frac": exact_bytes / (exact_ms * 1e-3) / 8.0e12,
            "decorr_exact_samples_per_s": samples / (exact_ms * 1e-3),
            "psf_from_sinc_ms": psf_ms}


def time_windows_fullw(pk, torch, ps, obs, dobs, src, prec, ws, reps=5):
    """Windowed averaging (tapered baseline-dependent windows on both axes)
    and the exact-w patch on the same workload and source."""
    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    dw = pk.DeviceObservation(ps.tapered_windows(obs))
    D = torch.empty((dobs.K, 2), dtype=torch.float32, device="cuda")
    win = {"decorr_windowed_ms": timed(lambda: pk.decorr(dw, src.l0, src.m0, out=D)),
           "decorr_boxcar_ms": timed(lambda: pk.decorr(dobs, src.l0, src.m0, out=D)),
           "psf_windowed_ms": timed(lambda: pk.patch(dw, src, prec=prec, workspace=ws))}
    del dw
    out = torch.empty((src.nl, src.nm), dtype=torch.float32, device="cuda")
    n_terms = pk.patch_fullw(dobs, src, prec=prec, out=out, workspace=ws)[1]
    torch.cuda.synchronize()  # the warm-up's contractions are still queued when it returns
    t0 = time.perf_counter()
    for _ in range(reps):
        pk.patch_fullw(dobs, src, prec=prec, out=out, workspace=ws)
    torch.cuda.synchronize()
    fullw = {"ms": (time.perf_counter() - t0) / reps * 1e3, "contractions": n_terms}
    return win, fullw


def time_method2(pk, torch, ps, dobs, src, prec, ws, N=256, n_src=16, reps=10):
    """The paper's Method 2 on the same workload: the effective PSF and its
    spectrum on an N x N grid at the patch's cell (once), then n_src
    per-source patches from it (fringe-rate D^ product and inverse FFT)."""
    cell = src.dl
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = pk.method2_spectrum(dobs, N, cell, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    spec_ms = (time.perf_counter() - t0) * 1e3
    dirs = [(src.l0 + 1e-3 * q, src.m0 - 5e-4 * q) for q in range(n_src)]
    out = torch.empty((n_src, N, N), dtype=torch.float32, device="cuda")
    pk.method2_patches(S, cell, dirs, 20.0, 2.5e7, 1.4e9, out=out, workspace=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pk.method2_patches(S, cell, dirs, 20.0, 2.5e7, 1.4e9, out=out, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    per = e0.elapsed_time(e1) / reps / n_src
    return {"grid": [N, N], "spectrum_ms": spec_ms, "per_source_ms": per, "sources_per_s": 1e3 / per,
            "batch": n_src}


def time_adjoint(pk, torch, ps, dobs, prec, ws, reps=3):
    """The differentiation workload on the same data: 16 sources at 0.2-2 deg
    with 129 x 129 patches, one batched forward and one adjoint call
    (d/d(l0, m0) of every source from a cotangent of all 16 patches)."""
    srcs = ps.sources(3, seed=0)
    n = sum(s.nl * s.nm for s in srcs)
    G = torch.randn(n, dtype=torch.float32, device="cuda")
    pk.patch_batched(dobs, srcs, prec=prec, workspace=ws)
    pk.patch_backward(dobs, srcs, G, prec, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        pk.patch_batched(dobs, srcs, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        pk.patch_backward(dobs, srcs, G, prec, workspace=ws)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fwd, bwd = (t1 - t0) / reps * 1e3, (t2 - t1) / reps * 1e3
    return {"sources": len(srcs), "patch": [srcs[0].nl, srcs[0].nm], "forward_ms": fwd, "backward_ms": bwd,
            "backward_over_forward": bwd / fwd}


def time_clean(pk, torch, ps, dobs, grid, prec, ws, cycles=20):
    """Hogbom CLEAN with the distorted PSF at every peak on a 257 x 257 image
    of this workload: three sources placed on pixels, dirty image formed by
    the library, `cycles` minor cycles timed (each one PSF evaluation plus
    the peak search, subtraction and one read-back), then the same cycles
    kept on the device and replayed from a captured graph."""
    dirty = torch.zeros((grid.nl, grid.nm), dtype=torch.float32, device="cuda")
    for i, j, f in ((60, 70, 1.0), (180, 150, 0.5), (128, 230, 0.25)):
        s = grid.with_direction(grid.l_first + i * grid.dl, grid.m_first + j * grid.dm)
        dirty += f * pk.patch(dobs, s, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, comps = pk.clean_hogbom(dobs, grid, dirty, cycles, 0.1, 0.0, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same cycles kept on the device (no read-back), captured once and replayed
    res = dirty.clone()
    cc = pk.clean_hogbom_device(dobs, grid, res, cycles, 0.1, 0.0, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pk.clean_hogbom_device(dobs, grid, res, cycles, 0.1, 0.0, prec=prec, workspace=ws, comps=cc)
    res.copy_(dirty)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.replay()
    torch.cuda.synchronize()
    dt_dev = time.perf_counter() - t0
    del g
    # the same image with Method-2 PSFs (512 x 512 spectrum: covers the image from any peak)
    S = pk.method2_spectrum(dobs, 512, grid.dl, prec=prec, workspace=ws)
    pk.clean_hogbom_method2(S, grid, dirty, 2, 20.0, 2.5e7, 1.4e9, 0.1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, comps2 = pk.clean_hogbom_method2(S, grid, dirty, 10 * cycles, 20.0, 2.5e7, 1.4e9, 0.1)
    torch.cuda.synchronize()
    dt2 = time.perf_counter() - t0
    # the Method-2 cycles kept on the device, captured once and replayed
    res2 = dirty.clone()
    cc2 = pk.clean_hogbom_method2_device(S, grid, res2, 10 * cycles, 20.0, 2.5e7, 1.4e9, 0.1)
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2):
        pk.clean_hogbom_method2_device(S, grid, res2, 10 * cycles, 20.0, 2.5e7, 1.4e9, 0.1, comps=cc2)
    res2.copy_(dirty)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g2.replay()
    torch.cuda.synchronize()
    dt2_dev = time.perf_counter() - t0
    del g2
    return {"image": [grid.nl, grid.nm], "cycles": len(comps), "ms_per_cycle": dt / max(1, len(comps)) * 1e3,
            "device_graph_ms_per_cycle": dt_dev / cycles * 1e3,
            "method2_psf_grid": [512, 512], "method2_cycles": len(comps2),
            "method2_ms_per_cycle": dt2 / max(1, len(comps2)) * 1e3,
            "method2_device_graph_ms_per_cycle": dt2_dev / (10 * cycles) * 1e3}


GOLD = os.path.join(ROOT, "tests", "golden")


def golden_pixels(names):
    """Stored FP64 oracle values at sampled pixels: {source index: (i, j,
    P_ij, scale)} from the listed golden files that exist; scale is the
    error's normaliser, max |P64| over the patch bounded below by the stored
    pixels and the value at the source."""
    import numpy as np
    out = {}
    for n in names:
        f = os.path.join(GOLD, n)
        if not os.path.exists(f):
            continue
        rows = np.load(f)
        for i in np.unique(rows[:, 0]).astype(int):
            sel = rows[:, 0] == i
            # normaliser: max |P64| over the patch, bounded below by the stored pixels and the source's value
            out[int(i)] = (rows[sel, 1].astype(int), rows[sel, 2].astype(int), rows[sel, 3],
                           max(abs(rows[sel, 4][0]), float(np.max(np.abs(rows[sel, 3])))))
    return out


def headline_bda(pk, torch, ps, obs, srcs, prec, steps, warmup, ws, per_slice=16):
    """One graph per 16-source slice of the headline workload, each holding
    one psf_patch_batched call; `steps` replays cycling through the slices
    are timed.  Returns the line's timing fields, the roofline of the
    contraction kernel from an eager pass over every slice with HIP events
    on its launch stream, and the error of the timed output at the stored
    oracle pixels."""
    import numpy as np
    dobs = pk.DeviceObservation(obs)
    slices = [srcs[i:i + per_slice] for i in range(0, len(srcs), per_slice)]
    need = max(pk.workspace_bytes(dobs, sl, prec) for sl in slices)
    ws.get(need)
    # load every tile family's kernels once, outside capture
    first = []
    for n in sorted({s.nl for s in srcs}):
        first.append(next(s for s in srcs if s.nl == n))
    pk.patch_batched(dobs, first, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    graphs, outs, terms = [], [], []
    for sl in slices:
        _, d = pk.device_sources(sl, dobs.device)
        out = torch.empty(sum(s.nl * s.nm for s in sl), dtype=torch.float32, device="cuda")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            pk.patch_batched(dobs, sl, prec=prec, out=out, workspace=ws, d_srcs=d)
        graphs.append((g, d))
        outs.append(out)
        terms.append(float(dobs.K) * sum(s.nl * s.nm for s in sl))
    torch.cuda.synchronize()
    for w in range(warmup):
        graphs[w % len(graphs)][0].replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0.0
    for st in range(steps):
        q = st % len(graphs)
        graphs[q][0].replay()
        done += terms[q]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"headline: {steps} replays in {wall:.1f} s", file=sys.stderr, flush=True)
    # error of what the timed replays wrote, at the stored oracle pixels
    gold = golden_pixels(["config5_seed0_pixels.npy", "config5_seed0_far_pixels.npy"])
    errs = {}
    for i, (ii, jj, ref, peak) in sorted(gold.items()):
        q, r = divmod(i, per_slice)
        if q >= min(steps, len(graphs)) and q >= warmup:
            continue
        P = pk.split_patches(outs[q], slices[q])[r].cpu().numpy().astype(np.float64)
        errs[str(i)] = float(np.max(np.abs(P[ii, jj] - ref)) / abs(peak))
    # the contraction kernel's launches, timed with events on its stream
    pk.psf_timing_read()
    pk.psf_timing_enable(True)
    t1 = time.perf_counter()
    for sl in slices:
        pk.patch_batched(dobs, sl, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    eager_s = time.perf_counter() - t1
    kms, nk = pk.psf_timing_read()
    pk.psf_timing_enable(False)
    all_terms = float(sum(terms))
    del graphs, outs, dobs
    torch.cuda.empty_cache()
    return {"ms_per_step": wall / steps * 1e3, "terms_per_s": done / wall,
            "psfs_per_s": steps * per_slice / wall, "graph_replays": steps,
            "eager_all_256_s": eager_s, "kernel_ms_total": kms, "kernel_launches": nk,
            "all_terms": all_terms, "errors": errs,
            "slices": len(slices), "sizes": {str(n): sum(1 for s in srcs if s.nl == n)
                                             for n in sorted({s.nl for s in srcs})}}


SYM_SIZES = {(257, 17), (129, 9), (65, 5)}  # (rows, column blocks) with the symmetric form


def executed_flops(K, srcs, prec):
    """Matrix-core flops the contraction executes for these patches: per
    visibility (16 nbi) x (16 nbj) multiply-adds over one real inner value in
    the symmetric form (C and S rows of 16-row blocks), two (re, im) in the
    general form, times the split products."""
    tot = 0.0
    for s in srcs:
        nbi, nbj = (s.nl + 15) // 16, (s.nm + 15) // 16
        sym = (s.nl, nbj) in SYM_SIZES
        inner = 1 if sym else 2
        prods = PRODUCTS[prec]
        if prec in ("mixed_fp16", "sr_fp16") and not (sym and K >= MIXED_MIN_K):
            prods = PRODUCTS["split_fp16"]
        tot += float(K) * inner * (16 * nbi) * (16 * nbj) * 2.0 * prods
    return tot


def roofline(prec, terms, kernel_ms, launches, traffic=None, kernel="k_patch", exec_flops=None):
    """Useful matrix-core work (4 flops per term) per launch over the
    kernel's average launch time, against the dense peak of its arithmetic;
    the executed work (split products, the symmetric form and tile padding
    counted) beside it."""
    per_launch_ms = kernel_ms / max(launches, 1)
    per_launch_flops = ALG_FLOPS_PER_TERM * terms / max(launches, 1)
    achieved = per_launch_flops / (per_launch_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    out = {"bound": "mfma", "kernel": f"{kernel}<{prec}>", "achieved": achieved, "peak": peak,
           "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
           "kernel_ms": per_launch_ms, "launches": launches,
           "per_unit": f"{ALG_FLOPS_PER_TERM:g} flops per useful one-sided term (2 real multiply-adds), "
                       f"{terms / max(launches, 1):.4g} terms per launch on average"}
    if exec_flops is not None:
        out["frac_executed"] = exec_flops / max(launches, 1) / (per_launch_ms * 1e-3) / 1e12 / peak
    return out


def precision_workload(pk, torch, ps, ws, seed=0):
    """The precision workload (K = 23.2M, 64 sources of 257^2 at 0.1-3 deg),
    each arithmetic in one batched call: time, terms/s and the error at the
    stored oracle pixels (twelve sources)."""
    import numpy as np
    obs = ps.observation(4, seed=seed)
    srcs = ps.sources(4, seed=seed)
    dobs = pk.DeviceObservation(obs)
    terms = float(obs.K) * sum(s.nl * s.nm for s in srcs)
    gold = golden_pixels(["config4_seed0_pixels.npy", "config4_seed0_more_pixels.npy"])
    out = {"workload": "64 antennas, 1800 x 2 s, 64 ch over 0.9-1.7 GHz, 10 s x 2 ch bins (K=23,224,320), "
                       "64 sources at 0.1-3 deg, 257x257 at 1.5 arcsec", "K": obs.K, "sources": len(srcs)}
    for prec in ("split_bf16", "split_fp16", "mixed_fp16", "sr_fp16", "fp32"):
        P = pk.patch_batched(dobs, srcs, prec=prec, workspace=ws)
        torch.cuda.synchronize()
        pk.psf_timing_read()
        pk.psf_timing_enable(True)
        t0 = time.perf_counter()
        P = pk.patch_batched(dobs, srcs, prec=prec, workspace=ws, out=P)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kms, nk = pk.psf_timing_read()
        pk.psf_timing_enable(False)
        parts = pk.split_patches(P, srcs)
        err = max((float(np.max(np.abs(parts[i].cpu().numpy().astype(np.float64)[ii, jj] - ref)) / abs(peak))
                   for i, (ii, jj, ref, peak) in gold.items()), default=None)
        out[prec] = {"s": dt, "terms_per_s": terms / dt, "psfs_per_s": len(srcs) / dt,
                     "contraction_tflops_useful": ALG_FLOPS_PER_TERM * terms / (kms * 1e-3) / 1e12,
                     "frac_useful": ALG_FLOPS_PER_TERM * terms / (kms * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
                     "max_err_at_oracle_pixels": err}
    out["split_bf16_over_fp32"] = out["fp32"]["s"] / out["split_bf16"]["s"]
    del dobs
    torch.cuda.empty_cache()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(obs, src, n_bl_sub):
    """The FP64 oracle (decorr + factored patch) for one source on the first
    n_bl_sub baselines of the workload."""
    import numpy as np

    import oracle as orc
    import psf_synth as ps
    B = min(n_bl_sub, obs.n_bl)
    k1 = int(obs.bl_koff[B])
    sub = ps.first_baselines(obs, B)
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        blas_threads = None
    t0 = time.perf_counter()
    D = orc.decorr(sub, src.l0, src.m0)
    P = orc.patch_factored(sub, src, D)
    dt = time.perf_counter() - t0
    assert np.isfinite(P).all()
    terms = k1 * src.nl * src.nm
    return {"value": terms / dt, "unit": "terms/s", "cores": blas_threads or len(os.sched_getaffinity(0)),
            "kind": "oracle",
            "sample": f"FP64 oracle decorr + factored patch of one {src.nl}x{src.nm} source over the first {B} "
                      f"of {obs.n_bl} baselines of the headline workload ({k1} of {obs.K} bins), {dt:.1f} s; "
                      f"host has {len(os.sched_getaffinity(0))} usable cores",
            "cpu_model": cpu_model(), "host_cores": len(os.sched_getaffinity(0)), "blas_threads": blas_threads}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); multi-GPU sharding is not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2009_07010_amd as pk
    import psf_synth as ps
    assert torch.cuda.is_available(), "needs a GPU"
    ws = pk.Workspace()

    if a.copy_mib > 0:
        n = a.copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(f"copied {a.copy_mib} MiB 3 times", flush=True)
        return

    if a.profile_steps > 0 and a.profile_workload != "bda256":
        cfg = 5 if a.profile_workload == "decorr-bda" else 2
        obs = ps.observation(cfg, seed=a.seed)
        src = ps.sources(cfg, seed=a.seed)[0]
        dobs = pk.DeviceObservation(obs)
        if a.profile_workload == "forward129":
            srcs = ps.sources(3, seed=a.seed)
            for _ in range(a.profile_steps):
                pk.patch_batched(dobs, srcs, a.prec, workspace=ws)
        elif a.profile_workload == "adjoint129":
            srcs = ps.sources(3, seed=a.seed)
            G = torch.randn(sum(s.nl * s.nm for s in srcs), dtype=torch.float32, device="cuda")
            for _ in range(a.profile_steps):
                pk.patch_backward(dobs, srcs, G, a.prec, workspace=ws)
        elif a.profile_workload.startswith("decorr"):
            # the decorrelation as the patch path runs it (factors, records and
            # W D written per bin), here ahead of a small 65 x 65 contraction
            small = ps.Source.centred(src.l0, src.m0, 65, src.dl)
            for _ in range(a.profile_steps):
                pk.patch(dobs, small, prec=a.prec, workspace=ws)
        else:
            for _ in range(a.profile_steps):
                pk.patch(dobs, src, prec=a.prec, workspace=ws)
        torch.cuda.synchronize()
        print(f"profiled {a.profile_steps} steps of {a.profile_workload} ({a.prec})", flush=True)
        return

    print("generating the headline workload", file=sys.stderr, flush=True)
    obs5 = ps.observation(5, seed=a.seed)
    srcs5 = ps.sources(5, seed=a.seed)
    if a.profile_steps > 0:
        h = headline_bda(pk, torch, ps, obs5, srcs5, a.prec, a.profile_steps, 1, ws)
        print(f"profiled {a.profile_steps} headline steps of {a.prec}: {h['ms_per_step']:.1f} ms/step", flush=True)
        return
    print("timing the headline workload", file=sys.stderr, flush=True)
    h = headline_bda(pk, torch, ps, obs5, srcs5, a.prec, a.steps, a.warmup, ws)
    rf = roofline(a.prec, h["all_terms"], h["kernel_ms_total"], h["kernel_launches"],
                  measured_traffic(a.prec, "bda256"), exec_flops=executed_flops(obs5.K, srcs5, a.prec))
    line = {
        "metric": "PSF vis·pixel terms/s at ≤1e-5 rel err vs FP64; PSFs/s, split-BF16 vs FP32",
        "value": h["terms_per_s"],
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[a.prec],
        "data": "synthetic",
        "config": {"workload": "baseline-dependent averaging, MeerKAT-shaped: 64 antennas (2016 baselines), "
                               "14400 x 1 s, 64 ch over 1.3-1.5 GHz, bins floor(B_max/|b|) clamped to 1-64 "
                               "samples x 1-8 ch, 256 sources at 0.05-3 deg with 65/129/257-pixel patches at "
                               "1.5 arcsec; one step = one graph replay of a 16-source psf_patch_batched call",
                   "K": obs5.K, "sources": len(srcs5), "patch_sizes": h["sizes"], "precision": a.prec,
                   "seed": a.seed},
        "psfs_per_s": h["psfs_per_s"],
        "max_rel_err_vs_fp64": max(h["errors"].values()) if h["errors"] else None,
        "errors_at_oracle_pixels": h["errors"],
        "all_256_eager_s": h["eager_all_256_s"],
        "roofline": rf,
    }
    if a.prec != "split_bf16":
        print("headline in split-BF16", file=sys.stderr, flush=True)
        hb = headline_bda(pk, torch, ps, obs5, srcs5, "split_bf16", 16, 2, ws)
        line["headline_split_bf16"] = {
            "ms_per_step": hb["ms_per_step"], "terms_per_s": hb["terms_per_s"], "psfs_per_s": hb["psfs_per_s"],
            "steps": 16, "warmup": 2, "max_rel_err_vs_fp64": max(hb["errors"].values()) if hb["errors"] else None,
            "errors_at_oracle_pixels": hb["errors"],
            "roofline": roofline("split_bf16", hb["all_terms"], hb["kernel_ms_total"], hb["kernel_launches"],
                                 measured_traffic("split_bf16", "bda256"),
                                 exec_flops=executed_flops(obs5.K, srcs5, "split_bf16"))}
    print("uniform-bin workload", file=sys.stderr, flush=True)
    obs = ps.observation(2, seed=a.seed)
    src = ps.sources(2, seed=a.seed)[0]
    dobs = pk.DeviceObservation(obs)
    terms = obs.K * src.nl * src.nm
    ms, kms, _ = time_prec(pk, torch, dobs, src, a.prec, a.steps, a.warmup, ws)
    ms32, kms32, _ = time_prec(pk, torch, dobs, src, "fp32", max(3, a.steps // 4), 1, ws)
    msb, kmsb, _ = time_prec(pk, torch, dobs, src, "split_bf16", a.steps, a.warmup, ws)
    line["meerkat257"] = {
        "workload": "64 antennas (2016 baselines), 3600 x 2 s, 32 ch over 1.3-1.5 GHz, 20 s x 4 ch bins "
                    "(K=5,806,080), 1 source at 1 deg, 257x257 at 1.5 arcsec, one psf_patch call per PSF",
        "K": obs.K, "terms_per_s": terms / (ms * 1e-3), "ms_per_psf": ms, "psfs_per_s": 1e3 / ms,
        "roofline": roofline(a.prec, float(terms), kms, 1, measured_traffic(a.prec),
                             exec_flops=executed_flops(obs.K, [src], a.prec)),
        "fp32": {"ms_per_psf": ms32, "terms_per_s": terms / (ms32 * 1e-3),
                 "roofline": roofline("fp32", float(terms), kms32, 1,
                                      exec_flops=executed_flops(obs.K, [src], "fp32"))},
        "split_bf16": {"ms_per_psf": msb, "terms_per_s": terms / (msb * 1e-3),
                       "roofline": roofline("split_bf16", float(terms), kmsb, 1, measured_traffic("split_bf16"),
                                            exec_flops=executed_flops(obs.K, [src], "split_bf16"))}}
    print("extras", file=sys.stderr, flush=True)
    line["method1"] = time_method1(pk, torch, dobs, src, a.prec, ws)
    line["clean"] = time_clean(pk, torch, ps, dobs, src, a.prec, ws)
    line["windows"], line["fullw"] = time_windows_fullw(pk, torch, ps, obs, dobs, src, a.prec, ws)
    line["method2"] = time_method2(pk, torch, ps, dobs, src, a.prec, ws)
    line["adjoint"] = time_adjoint(pk, torch, ps, dobs, a.prec, ws)
    del dobs
    torch.cuda.empty_cache()
    print("precision workload", file=sys.stderr, flush=True)
    line["precision"] = precision_workload(pk, torch, ps, ws, a.seed)
    if not a.no_cpu_baseline:
        print("CPU reference", file=sys.stderr, flush=True)
        src_c = next(s for s in srcs5 if s.nl == 129)
        cb = cpu_baseline(obs5, src_c, a.cpu_baselines)
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
