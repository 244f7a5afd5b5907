"""Write stored expected values for the full-size GPU parity tests.

Calls only the FP64 CPU reference (``oracle``) on inputs from the seeded
generator (``psf_synth``); nothing here touches the GPU library.

    python tests/golden/make_golden.py [config2] [config3] ...
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as orc  # noqa: E402
import psf_synth as ps  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _meta(name, **kw):
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(kw, f, indent=1)


def config2():
    obs = ps.observation(2, seed=0)
    src = ps.sources(2, seed=0)[0]
    t = time.time()
    D = orc.decorr(obs, src.l0, src.m0)
    td = time.time() - t
    P = orc.patch_factored(obs, src, D)
    tp = time.time() - t - td
    np.save(os.path.join(HERE, "config2_seed0_P.npy"), P)
    ks = np.random.default_rng(0).choice(obs.K, 4096, replace=False)
    np.save(os.path.join(HERE, "config2_seed0_Dsample.npy"), np.stack([ks, D[ks].real, D[ks].imag], axis=1))
    _meta("config2_seed0", config=2, seed=0, K=obs.K, l0=src.l0, m0=src.m0, nl=src.nl, nm=src.nm,
          decorr_s=td, patch_s=tp, what="oracle.patch_factored (FP64) of workload 2, seed 0")
    print("config2", td, tp)


def _config3(obs, tag, n_src):
    """Differentiation workload: the first n_src sources of workload 3, targets
    flux * P at positions perturbed by N(0, 1 arcsec) per axis (same grid),
    rounded to float32 as the GPU test feeds them, and the FP64 loss and
    gradients for those targets."""
    srcs = ps.sources(3, seed=0)[:n_src]
    moved = ps.perturbed_targets(3, srcs, seed=0)
    t = time.time()
    T = np.stack([s.flux * orc.patch_factored(obs, m) for s, m in zip(srcs, moved)]).astype(np.float32)
    fluxes = [s.flux for s in srcs]
    L, g_lm, g_f = orc.loss_grad_analytic(obs, srcs, fluxes, [x.astype(np.float64) for x in T])
    np.save(os.path.join(HERE, f"{tag}_targets.npy"), T)
    np.save(os.path.join(HERE, f"{tag}_grad.npy"), np.concatenate([g_lm, g_f[:, None]], axis=1))
    _meta(tag, config=3, seed=0, n_src=n_src, n_bl=obs.n_bl, K=obs.K, loss=L, seconds=time.time() - t,
          what="oracle.loss_grad_analytic (FP64): columns dL/dl0, dL/dm0, dL/dflux per source; "
               "targets from oracle.patch_factored at the perturbed positions, float32")
    print(tag, time.time() - t)


def _config3_flux_scale(obs, tag):
    """sum_ij |2 r_ij P_ij| per source (r = flux P - T): the magnitude of the
    terms of dL/dflux, which cancel near the optimum; the scale the flux
    derivative's error is measured against."""
    meta = json.load(open(os.path.join(HERE, tag + ".json")))
    srcs = ps.sources(3, seed=0)[:meta["n_src"]]
    T = np.load(os.path.join(HERE, tag + "_targets.npy")).astype(np.float64)
    out = []
    for s, t in zip(srcs, T):
        P = orc.patch_factored(obs, s)
        out.append(2.0 * np.sum(np.abs((s.flux * P - t) * P)))
    np.save(os.path.join(HERE, tag + "_fluxscale.npy"), np.array(out))
    print(tag, "flux scale", out)


def config3_sub_fluxscale():
    _config3_flux_scale(ps.first_baselines(ps.observation(3, seed=0), 64), "config3_seed0_bl64")


def config3_fluxscale():
    _config3_flux_scale(ps.observation(3, seed=0), "config3_seed0")


def config3_sub():
    _config3(ps.first_baselines(ps.observation(3, seed=0), 64), "config3_seed0_bl64", 4)


def config3():
    _config3(ps.observation(3, seed=0), "config3_seed0", 4)


def config5_pixels(srcs, n_side):
    """Sampled pixels of a patch: the centre, the four corners, edge
    midpoints and seeded random pixels (row, column indices)."""
    out = []
    for s in srcs:
        nl, nm = s.nl, s.nm
        fixed = [(nl // 2, nm // 2), (0, 0), (0, nm - 1), (nl - 1, 0), (nl - 1, nm - 1),
                 (nl // 2, 0), (0, nm // 2), (nl - 1, nm // 2), (nl // 2, nm - 1)]
        g = np.random.default_rng(5)
        rnd = [(int(g.integers(nl)), int(g.integers(nm))) for _ in range(n_side - len(fixed))]
        ij = np.array(fixed + rnd)
        out.append(ij)
    return out


def config5_sources():
    """One source of each patch size of workload 5: the first of each size."""
    srcs = ps.sources(5, seed=0)
    idx = []
    for n in (65, 129, 257):
        idx.append(next(i for i, s in enumerate(srcs) if s.nl == n))
    return idx


def config5():
    obs = ps.observation(5, seed=0)
    srcs = ps.sources(5, seed=0)
    idx = config5_sources()
    pix = config5_pixels([srcs[i] for i in idx], 24)
    t = time.time()
    rows = []
    for i, ij in zip(idx, pix):
        D = orc.decorr(obs, srcs[i].l0, srcs[i].m0)
        P = orc.patch_pixels(obs, srcs[i], ij[:, 0], ij[:, 1], D)
        peak = 2.0 * float(np.sum(obs.W.astype(np.float64) * D.real))
        for (a, b), v in zip(ij, P):
            rows.append((i, a, b, v, peak))
        print("config5 source", i, time.time() - t, flush=True)
    np.save(os.path.join(HERE, "config5_seed0_pixels.npy"), np.array(rows, dtype=np.float64))
    _meta("config5_seed0", config=5, seed=0, K=obs.K, sources=idx, seconds=time.time() - t,
          what="oracle.patch_pixels (FP64) at sampled pixels of one source per patch size of workload 5; "
               "columns: source index, i, j, P_ij, peak 2 Re sum W D")


def config5_far_sources():
    """The source of each patch size of workload 5 at the largest radius
    (where the phase factors turn fastest and the split forms' errors peak)."""
    srcs = ps.sources(5, seed=0)
    idx = []
    for n in (65, 129, 257):
        cand = [i for i, s in enumerate(srcs) if s.nl == n]
        idx.append(max(cand, key=lambda i: np.hypot(srcs[i].l0, srcs[i].m0)))
    return idx


def config5_far():
    """Workload 5 at sampled pixels of the largest-radius source of each
    patch size (65, 129, 257), FP64, with each patch's peak."""
    obs = ps.observation(5, seed=0)
    srcs = ps.sources(5, seed=0)
    idx = config5_far_sources()
    pix = config5_pixels([srcs[i] for i in idx], 24)
    t = time.time()
    rows = []
    for i, ij in zip(idx, pix):
        D = orc.decorr(obs, srcs[i].l0, srcs[i].m0)
        P = orc.patch_pixels(obs, srcs[i], ij[:, 0], ij[:, 1], D)
        peak = 2.0 * float(np.sum(obs.W.astype(np.float64) * D.real))
        rows += [(i, a, b, v, peak) for (a, b), v in zip(ij, P)]
        print("config5 far source", i, time.time() - t, flush=True)
    np.save(os.path.join(HERE, "config5_seed0_far_pixels.npy"), np.array(rows, dtype=np.float64))
    _meta("config5_seed0_far", config=5, seed=0, K=obs.K, sources=idx,
          radii_deg=[float(np.degrees(np.arcsin(np.hypot(srcs[i].l0, srcs[i].m0)))) for i in idx],
          seconds=time.time() - t,
          what="oracle.patch_pixels (FP64) at sampled pixels of the largest-radius source of each patch "
               "size of workload 5; columns: source index, i, j, P_ij, peak 2 Re sum W D")


CONFIG4_SOURCES = [5, 7, 0, 2]    # radii 0.45, 1.67, 1.87, 2.8 deg


def config4():
    """The precision workload (K = 23.2M, 257 x 257 patches): FP64 values at
    20 sampled pixels of four of its 64 sources, with each patch's peak."""
    obs = ps.observation(4, seed=0)
    srcs = ps.sources(4, seed=0)
    pix = config5_pixels([srcs[i] for i in CONFIG4_SOURCES], 20)
    t = time.time()
    rows = []
    for i, ij in zip(CONFIG4_SOURCES, pix):
        D = orc.decorr(obs, srcs[i].l0, srcs[i].m0)
        P = orc.patch_pixels(obs, srcs[i], ij[:, 0], ij[:, 1], D)
        peak = 2.0 * float(np.sum(obs.W.astype(np.float64) * D.real))
        rows += [(i, a, b, v, peak) for (a, b), v in zip(ij, P)]
        print("config4 source", i, time.time() - t, flush=True)
    np.save(os.path.join(HERE, "config4_seed0_pixels.npy"), np.array(rows, dtype=np.float64))
    _meta("config4_seed0", config=4, seed=0, K=obs.K, sources=CONFIG4_SOURCES, seconds=time.time() - t,
          what="oracle.patch_pixels (FP64) at sampled pixels of four sources of workload 4; "
               "columns: source index, i, j, P_ij, peak 2 Re sum W D")


CONFIG4_MORE_SOURCES = [20, 41, 53, 21, 56, 12, 34, 54]    # radii 0.2, 1.04, 2.36, 2.57, 2.94, 2.95, 2.95, 2.96 deg


def config4_more():
    """Workload 4: FP64 values at 20 sampled pixels of eight more of its 64
    sources (the nearest, one at 1 deg and the farthest six, where the split
    forms' errors are largest), with each patch's peak."""
    obs = ps.observation(4, seed=0)
    srcs = ps.sources(4, seed=0)
    pix = config5_pixels([srcs[i] for i in CONFIG4_MORE_SOURCES], 20)
    t = time.time()
    rows = []
    for i, ij in zip(CONFIG4_MORE_SOURCES, pix):
        D = orc.decorr(obs, srcs[i].l0, srcs[i].m0)
        P = orc.patch_pixels(obs, srcs[i], ij[:, 0], ij[:, 1], D)
        peak = 2.0 * float(np.sum(obs.W.astype(np.float64) * D.real))
        rows += [(i, a, b, v, peak) for (a, b), v in zip(ij, P)]
        print("config4 source", i, time.time() - t, flush=True)
    np.save(os.path.join(HERE, "config4_seed0_more_pixels.npy"), np.array(rows, dtype=np.float64))
    _meta("config4_seed0_more", config=4, seed=0, K=obs.K, sources=CONFIG4_MORE_SOURCES, seconds=time.time() - t,
          what="oracle.patch_pixels (FP64) at sampled pixels of eight more sources of workload 4; "
               "columns: source index, i, j, P_ij, peak 2 Re sum W D")


def config2_windows():
    """Workload 2 with the tapered baseline-dependent windows of
    ``psf_synth.tapered_windows`` (strength 1): sampled D and sampled pixels
    of the source's 257 x 257 patch, with the patch peak."""
    obs = ps.tapered_windows(ps.observation(2, seed=0))
    src = ps.sources(2, seed=0)[0]
    t = time.time()
    D = orc.decorr(obs, src.l0, src.m0)
    ks = np.random.default_rng(0).choice(obs.K, 4096, replace=False)
    np.save(os.path.join(HERE, "config2_seed0_win_Dsample.npy"), np.stack([ks, D[ks].real, D[ks].imag], axis=1))
    ij = config5_pixels([src], 48)[0]
    P = orc.patch_pixels(obs, src, ij[:, 0], ij[:, 1], D)
    peak = 2.0 * float(np.sum(obs.W.astype(np.float64) * D.real))
    np.save(os.path.join(HERE, "config2_seed0_win_pixels.npy"),
            np.concatenate([ij.astype(np.float64), P[:, None], np.full((len(P), 1), peak)], axis=1))
    _meta("config2_seed0_win", config=2, seed=0, K=obs.K, windows="tapered_windows(strength=1)",
          seconds=time.time() - t,
          what="oracle.decorr (windowed, FP64) at 4096 sampled bins: k, Re D, Im D; oracle.patch_pixels at "
               "sampled pixels: i, j, P_ij, peak 2 Re sum W D")
    print("config2_windows", time.time() - t)


def config2_fullw():
    """Workload 2's source patch (257 x 257 at 1.5 arcsec) with the exact w
    phase, at sampled pixels, with the linearised patch at the same pixels
    and the patch peak."""
    obs = ps.observation(2, seed=0)
    src = ps.sources(2, seed=0)[0]
    t = time.time()
    D = orc.decorr(obs, src.l0, src.m0)
    ij = config5_pixels([src], 48)[0]
    Pw = orc.patch_fullw_pixels(obs, src, ij[:, 0], ij[:, 1], D)
    Pl = orc.patch_pixels(obs, src, ij[:, 0], ij[:, 1], D)
    peak = 2.0 * float(np.sum(obs.W.astype(np.float64) * D.real))
    np.save(os.path.join(HERE, "config2_seed0_fullw_pixels.npy"),
            np.concatenate([ij.astype(np.float64), Pw[:, None], Pl[:, None], np.full((len(Pw), 1), peak)], axis=1))
    _meta("config2_seed0_fullw", config=2, seed=0, K=obs.K, seconds=time.time() - t,
          what="oracle.patch_fullw_pixels (FP64, exact w phase) at sampled pixels: i, j, P_full, "
               "P_linearised (oracle.patch_pixels), peak 2 Re sum W D")
    print("config2_fullw", time.time() - t)


if __name__ == "__main__":
    todo = sys.argv[1:] or ["config2"]
    for name in todo:
        globals()[name]()
