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


def config3_sub():
    _config3(ps.first_baselines(ps.observation(3, seed=0), 64), "config3_seed0_bl64", 4)


def config3():
    _config3(ps.observation(3, seed=0), "config3_seed0", 4)


if __name__ == "__main__":
    todo = sys.argv[1:] or ["config2"]
    for name in todo:
        globals()[name]()
