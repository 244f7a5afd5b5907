"""Throughput of the distorted-PSF hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec split_bf16]

One step = one PSF of the MeerKAT-shaped workload (64 antennas, 2016
baselines, 3600 x 2 s, 32 channels over 1.3-1.5 GHz, 20 s x 4 channel bins:
K = 5,806,080 averaged visibilities; one source at 1 deg; 257 x 257 patch at
1.5"): decorrelation factors, phase factors, contraction and finalise, all
inside one psf_patch call on device-resident inputs.  The value is
vis.pixel terms/s (K x 257^2 one-sided terms per PSF).

Printed: one JSON line with the headline (split-BF16 unless --prec says
otherwise), the same workload in plain FP32 for comparison, the roofline of
the contraction kernel measured with HIP events on its launch stream, and
the FP64 CPU reference timed on a bounded sample on this host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"split_bf16": 2516.6, "split_fp16": 2516.6, "plain_bf16": 2516.6, "fp32": 157.3}
# executed matrix-core flops per useful one-sided term: 2 real MACs (Re*Re and
# Im*Im) per term, times 3 products for the split forms
FLOPS_PER_TERM = {"split_bf16": 12.0, "split_fp16": 12.0, "plain_bf16": 4.0, "fp32": 4.0}
DTYPE = {"split_bf16": "bf16", "split_fp16": "fp16", "plain_bf16": "bf16", "fp32": "f32"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="split_bf16", choices=list(PEAK_TFLOPS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baselines", type=int, default=512,
                    help="baselines in the CPU-reference sample")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="if > 0: only run this many steps of --prec (for rocprofv3) and print nothing else")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="if > 0: only copy a buffer of this many MiB a few times (calibrates the HBM "
                         "byte counters against a plain copy kernel) and print nothing else")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_patch_traffic_meerkat257.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2009_07010_amd", "csrc", "k_patch.hip")


def measured_traffic(prec):
    """HBM bytes per contraction launch from the committed counter summary,
    or None when there is none for this precision or the kernel source has
    changed since the counters were taken."""
    import hashlib
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
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
    the peak search, subtraction and one read-back)."""
    dirty = torch.zeros((grid.nl, grid.nm), dtype=torch.float32, device="cuda")
    for i, j, f in ((60, 70, 1.0), (180, 150, 0.5), (128, 230, 0.25)):
        s = grid.with_direction(grid.l_first + i * grid.dl, grid.m_first + j * grid.dm)
        dirty += f * pk.patch(dobs, s, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, comps = pk.clean_hogbom(dobs, grid, dirty, cycles, 0.1, 0.0, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same image with Method-2 PSFs (512 x 512 spectrum: covers the image from any peak)
    S = pk.method2_spectrum(dobs, 512, grid.dl, prec=prec, workspace=ws)
    pk.clean_hogbom_method2(S, grid, dirty, 2, 20.0, 2.5e7, 1.4e9, 0.1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, comps2 = pk.clean_hogbom_method2(S, grid, dirty, 10 * cycles, 20.0, 2.5e7, 1.4e9, 0.1)
    torch.cuda.synchronize()
    dt2 = time.perf_counter() - t0
    return {"image": [grid.nl, grid.nm], "cycles": len(comps), "ms_per_cycle": dt / max(1, len(comps)) * 1e3,
            "method2_psf_grid": [512, 512], "method2_cycles": len(comps2),
            "method2_ms_per_cycle": dt2 / max(1, len(comps2)) * 1e3}


def cpu_baseline(obs, src, n_bl_sub):
    """The FP64 oracle (decorr + factored patch) on the first n_bl_sub baselines."""
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
            "sample": f"FP64 oracle decorr + factored patch over the first {B} of {obs.n_bl} baselines "
                      f"({k1} of {obs.K} bins) x {src.nl}x{src.nm} pixels, {dt:.1f} s; host has "
                      f"{len(os.sched_getaffinity(0))} usable cores"}


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
    obs = ps.observation(2, seed=a.seed)
    src = ps.sources(2, seed=a.seed)[0]
    dobs = pk.DeviceObservation(obs)
    ws = pk.Workspace()
    terms = obs.K * src.nl * src.nm

    if a.copy_mib > 0:
        n = a.copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(f"copied {a.copy_mib} MiB 3 times", flush=True)
        return

    if a.profile_steps > 0:
        for _ in range(a.profile_steps):
            pk.patch(dobs, src, prec=a.prec, workspace=ws)
        torch.cuda.synchronize()
        print(f"profiled {a.profile_steps} steps of {a.prec}", flush=True)
        return

    ms, kms, _ = time_prec(pk, torch, dobs, src, a.prec, a.steps, a.warmup, ws)
    ms32, kms32, _ = time_prec(pk, torch, dobs, src, "fp32", max(3, a.steps // 4), 1, ws)
    flops = FLOPS_PER_TERM[a.prec] * terms
    achieved = flops / (kms * 1e-3) / 1e12
    line = {
        "metric": "PSF vis\u00b7pixel terms/s at \u22641e-5 rel err vs FP64; PSFs/s, split-BF16 vs FP32",
        "value": terms / (ms * 1e-3),
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[a.prec],
        "data": "synthetic",
        "config": {"workload": "MeerKAT-shaped: 64 antennas (2016 baselines), 3600 x 2 s, 32 ch over "
                               "1.3-1.5 GHz, 20 s x 4 ch bins (K=5,806,080), 1 source at 1 deg, 257x257 "
                               "patch at 1.5 arcsec",
                   "K": obs.K, "patch": [src.nl, src.nm], "precision": a.prec, "seed": a.seed},
        "psfs_per_s": 1e3 / ms,
        "fp32": {"ms_per_step": ms32, "terms_per_s": terms / (ms32 * 1e-3),
                 "contraction_ms": kms32,
                 "contraction_tflops": 4.0 * terms / (kms32 * 1e-3) / 1e12},
        "roofline": {"bound": "mfma", "kernel": f"k_patch<{a.prec}>", "achieved": achieved,
                     "peak": PEAK_TFLOPS[a.prec], "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[a.prec],
                     "traffic": measured_traffic(a.prec), "kernel_ms": kms,
                     "per_unit": f"{FLOPS_PER_TERM[a.prec]:g} matrix-core flops per useful term, "
                                 f"{terms} terms per launch"},
    }
    line["method1"] = time_method1(pk, torch, dobs, src, a.prec, ws)
    line["clean"] = time_clean(pk, torch, ps, dobs, src, a.prec, ws)
    line["windows"], line["fullw"] = time_windows_fullw(pk, torch, ps, obs, dobs, src, a.prec, ws)
    line["method2"] = time_method2(pk, torch, ps, dobs, src, a.prec, ws)
    line["adjoint"] = time_adjoint(pk, torch, ps, dobs, a.prec, ws)
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(obs, src, a.cpu_baselines)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
