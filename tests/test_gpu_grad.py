"""GPU parity of the adjoint (psf_patch_backward behind the autograd
Function) against the FP64 oracle's analytic gradient and its central finite
differences.

The loss is the patch-fitting loss of the differentiation workload:
L = sum_s || f_s P_s(l0_s, m0_s) - T_s ||^2 on fixed grids.  Gradient parity
bar: 1e-4 relative, per source, to the largest of its two direction
components (and 1e-4 relative for the flux component).
"""
import json
import os

import numpy as np
import pytest

import oracle as orc
import psf_synth as ps

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")
GRAD_TOL = 1e-4
PRECS = ["fp32", "split_bf16", "split_fp16"]


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2009_07010_amd as pk
    pk.lib()
    return pk


def _gpu_loss_grad(pk, obs, srcs, fluxes, targets, prec):
    dobs = pk.DeviceObservation(obs)
    fn = pk.psf_patch_fn()
    lm = torch.tensor([[s.l0, s.m0] for s in srcs], dtype=torch.float64, requires_grad=True)
    f = torch.tensor(fluxes, dtype=torch.float32, device="cuda", requires_grad=True)
    T = torch.as_tensor(np.stack(targets), dtype=torch.float32, device="cuda")
    out = fn.apply(lm, f, dobs, srcs, prec)
    loss = ((out.double() - T.double()) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    return float(loss.detach()), lm.grad.numpy().copy(), f.grad.double().cpu().numpy()


def _check(g_lm, g_f, ref_lm, ref_f, label, flux_scale=None):
    """Direction components relative to the larger of the source's two; the
    flux component relative to itself, or to ``flux_scale[s]`` where given:
    the sum of the magnitudes of the terms of dL/dflux = 2 sum r P (FP64
    oracle), which cancel near the optimum, so that a patch error of 1e-6
    of its peak can exceed 1e-4 of the cancelled sum."""
    for s in range(len(ref_lm)):
        scale = np.max(np.abs(ref_lm[s]))
        err = np.max(np.abs(g_lm[s] - ref_lm[s])) / scale
        fs = abs(ref_f[s]) if flux_scale is None else flux_scale[s]
        ferr = abs(g_f[s] - ref_f[s]) / fs
        print(f"{label} src{s}: dir rel err {err:.2e}  (|grad| {scale:.3e}); flux rel err {ferr:.2e} "
              f"(plain {abs(g_f[s] - ref_f[s]) / abs(ref_f[s]):.2e})", flush=True)
        assert err <= GRAD_TOL, (label, s, g_lm[s], ref_lm[s])
        assert ferr <= GRAD_TOL, (label, s, g_f[s], ref_f[s])


def _config1_case():
    obs = ps.observation(1)
    base = ps.sources(1)[0]
    cell = 2.0 * ps.ARCSEC
    dirs = [(base.l0, base.m0), (-0.4 * ps.DEG, 0.7 * ps.DEG), (1.1 * ps.DEG, -0.2 * ps.DEG)]
    srcs = [ps.Source.centred(l0, m0, 65, cell) for l0, m0 in dirs]
    fluxes = [1.0, 0.3, 0.05]
    g = np.random.default_rng(7)
    moved = [s.with_direction(s.l0 + g.normal(0, ps.ARCSEC), s.m0 + g.normal(0, ps.ARCSEC)) for s in srcs]
    targets = [(f * orc.patch_factored(obs, m)).astype(np.float32) for f, m in zip(fluxes, moved)]
    return obs, srcs, fluxes, targets


@pytest.mark.parametrize("prec", PRECS)
def test_backward_config1_vs_oracle(pk, prec):
    """K = 420 only: the split-BF16 patch carries close to its per-term error
    bound here, and dL/dflux = 2 sum r P cancels, so the flux component is
    measured against the magnitude of its terms."""
    obs, srcs, fluxes, targets = _config1_case()
    T64 = [t.astype(np.float64) for t in targets]
    L_ref, g_ref, gf_ref = orc.loss_grad_analytic(obs, srcs, fluxes, T64)
    P64 = [orc.patch_factored(obs, s) for s in srcs]
    fscale = [2.0 * np.sum(np.abs((f * P - T) * P)) for f, P, T in zip(fluxes, P64, T64)]
    L, g_lm, g_f = _gpu_loss_grad(pk, obs, srcs, fluxes, targets, prec)
    assert abs(L - L_ref) <= 1e-3 * L_ref
    _check(g_lm, g_f, g_ref, gf_ref, f"config1 {prec}", flux_scale=fscale)


def test_backward_config1_vs_finite_differences(pk):
    """Against central differences (h = 1e-3 arcsec) of the FP64 oracle loss."""
    obs, srcs, fluxes, targets = _config1_case()
    T64 = [t.astype(np.float64) for t in targets]
    g_fd = orc.loss_grad_fd(obs, srcs, fluxes, T64)
    _, g_ref, gf_ref = orc.loss_grad_analytic(obs, srcs, fluxes, T64)
    _, g_lm, g_f = _gpu_loss_grad(pk, obs, srcs, fluxes, targets, "split_bf16")
    for s in range(len(srcs)):
        scale = np.max(np.abs(g_fd[s]))
        err = np.max(np.abs(g_lm[s] - g_fd[s])) / scale
        print(f"config1 FD src{s}: rel err {err:.2e}", flush=True)
        assert err <= GRAD_TOL


def _golden_case(tag, obs):
    meta = json.load(open(os.path.join(GOLD, tag + ".json")))
    srcs = ps.sources(3, seed=0)[:meta["n_src"]]
    T = np.load(os.path.join(GOLD, tag + "_targets.npy"))
    ref = np.load(os.path.join(GOLD, tag + "_grad.npy"))
    meta["flux_scale"] = np.load(os.path.join(GOLD, tag + "_fluxscale.npy"))
    return srcs, [s.flux for s in srcs], list(T), ref, meta


@pytest.mark.parametrize("prec", PRECS)
def test_backward_config3_first_64_baselines(pk, prec):
    obs = ps.first_baselines(ps.observation(3, seed=0), 64)
    srcs, fluxes, T, ref, meta = _golden_case("config3_seed0_bl64", obs)
    assert obs.K == meta["K"]
    L, g_lm, g_f = _gpu_loss_grad(pk, obs, srcs, fluxes, T, prec)
    assert abs(L - meta["loss"]) <= 1e-3 * meta["loss"]
    _check(g_lm, g_f, ref[:, :2], ref[:, 2], f"config3/64bl {prec}", flux_scale=meta["flux_scale"])


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "sr_fp16"])
def test_backward_config3_full(pk, prec):
    tag = "config3_seed0"
    if not os.path.exists(os.path.join(GOLD, tag + "_grad.npy")):
        pytest.skip("golden values for the full differentiation workload not generated")
    obs = ps.observation(3, seed=0)
    srcs, fluxes, T, ref, meta = _golden_case(tag, obs)
    assert obs.K == meta["K"]
    L, g_lm, g_f = _gpu_loss_grad(pk, obs, srcs, fluxes, T, prec)
    assert abs(L - meta["loss"]) <= 1e-3 * meta["loss"]
    _check(g_lm, g_f, ref[:, :2], ref[:, 2], f"config3 {prec}", flux_scale=meta["flux_scale"])


def test_backward_zero_cotangent_and_repeatability(pk):
    obs, srcs, fluxes, targets = _config1_case()
    dobs = pk.DeviceObservation(obs)
    n = sum(s.nl * s.nm for s in srcs)
    zero = pk.patch_backward(dobs, srcs, torch.zeros(n, device="cuda"), "split_bf16")
    assert torch.count_nonzero(zero).item() == 0
    G = torch.as_tensor(np.random.default_rng(3).standard_normal(n), dtype=torch.float32, device="cuda")
    a = pk.patch_backward(dobs, srcs, G, "split_bf16")
    b = pk.patch_backward(dobs, srcs, G, "split_bf16")
    assert torch.equal(a, b)


def test_backward_linear_in_cotangent(pk):
    """The adjoint is linear in G: grad(2 G1 - G2) = 2 grad(G1) - grad(G2)."""
    obs, srcs, _, _ = _config1_case()
    dobs = pk.DeviceObservation(obs)
    n = sum(s.nl * s.nm for s in srcs)
    g = np.random.default_rng(11)
    G1 = torch.as_tensor(g.standard_normal(n), dtype=torch.float32, device="cuda")
    G2 = torch.as_tensor(g.standard_normal(n), dtype=torch.float32, device="cuda")
    a = pk.patch_backward(dobs, srcs, G1, "fp32")
    b = pk.patch_backward(dobs, srcs, G2, "fp32")
    c = pk.patch_backward(dobs, srcs, 2 * G1 - G2, "fp32")
    scale = torch.max(torch.abs(a)) + torch.max(torch.abs(b))
    assert torch.max(torch.abs(c - (2 * a - b))) <= 1e-5 * scale


def test_backward_config3_sixteen_sources_match_single_calls(pk):
    """All 16 sources of the differentiation workload at full size (K = 5.8e6,
    129 x 129): the adjoint of one 16-source call equals 16 one-source calls
    with the same cotangent blocks."""
    obs = ps.observation(3, seed=0)
    srcs = ps.sources(3, seed=0)
    assert len(srcs) == 16
    dobs = pk.DeviceObservation(obs)
    n = srcs[0].nl * srcs[0].nm
    G = torch.as_tensor(np.random.default_rng(5).standard_normal(16 * n), dtype=torch.float32, device="cuda")
    ws = pk.Workspace()
    allg = pk.patch_backward(dobs, srcs, G, "split_bf16", workspace=ws).cpu().numpy()
    for s in range(16):
        one = pk.patch_backward(dobs, [srcs[s]], G[s * n:(s + 1) * n], "split_bf16", workspace=ws).cpu().numpy()
        assert np.array_equal(one[0], allg[s]), s
    assert np.all(np.isfinite(allg)) and np.all(np.abs(allg) > 0)


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16", "fp32"])
def test_backward_257_patches(pk, prec):
    """257 x 257 patches: the reverse-mode kernel splits the rows into three
    ranges (split forms), FP32 takes the five-patch form; both against the
    FP64 analytic gradient."""
    obs = ps.observation(1)
    cell = 1.0 * ps.ARCSEC
    srcs = [ps.Source.centred(0.6 * ps.DEG, -0.2 * ps.DEG, 257, cell),
            ps.Source.centred(-0.3 * ps.DEG, 0.9 * ps.DEG, 257, cell)]
    fluxes = [1.0, 0.4]
    g = np.random.default_rng(13)
    moved = [s.with_direction(s.l0 + g.normal(0, ps.ARCSEC), s.m0 + g.normal(0, ps.ARCSEC)) for s in srcs]
    T = [(f * orc.patch_factored(obs, m)).astype(np.float32) for f, m in zip(fluxes, moved)]
    T64 = [t.astype(np.float64) for t in T]
    L_ref, g_ref, gf_ref = orc.loss_grad_analytic(obs, srcs, fluxes, T64)
    P64 = [orc.patch_factored(obs, s) for s in srcs]
    fscale = [2.0 * np.sum(np.abs((f * P - t) * P)) for f, P, t in zip(fluxes, P64, T64)]
    L, g_lm, g_f = _gpu_loss_grad(pk, obs, srcs, fluxes, T, prec)
    assert abs(L - L_ref) <= 1e-3 * L_ref
    _check(g_lm, g_f, g_ref, gf_ref, f"257 {prec}", flux_scale=fscale)
    dobs = pk.DeviceObservation(obs)
    # a ragged 257 x 200 patch through the raw adjoint, cotangent from the oracle
    rag = ps.Source.centred(0.2 * ps.DEG, 0.5 * ps.DEG, 257, cell, nm=200)
    Tr = orc.patch_factored(obs, rag.with_direction(rag.l0 + ps.ARCSEC, rag.m0 - ps.ARCSEC))
    _, g_rag, _ = orc.loss_grad_analytic(obs, [rag], [1.0], [Tr])
    G = torch.as_tensor(2.0 * (orc.patch_factored(obs, rag) - Tr), dtype=torch.float32, device="cuda").reshape(-1)
    got = pk.patch_backward(dobs, [rag], G, prec).cpu().numpy()
    err = np.max(np.abs(got[0] - g_rag[0])) / np.max(np.abs(g_rag[0]))
    print(f"257x200 {prec}: dir rel err {err:.2e}", flush=True)
    assert err <= GRAD_TOL


@pytest.mark.parametrize("prec", ["split_bf16", "fp32"])
def test_backward_wide_patch_five_patch_form(pk, prec):
    """A patch wider than the reverse-mode kernel takes (300 columns) goes
    through the five derivative patches; against the FP64 gradient."""
    obs = ps.observation(1)
    src = ps.Source.centred(0.4 * ps.DEG, 0.1 * ps.DEG, 64, 1.5 * ps.ARCSEC, nm=300)
    T = orc.patch_factored(obs, src.with_direction(src.l0 - ps.ARCSEC, src.m0 + 0.5 * ps.ARCSEC))
    _, g_ref, _ = orc.loss_grad_analytic(obs, [src], [1.0], [T])
    G = torch.as_tensor(2.0 * (orc.patch_factored(obs, src) - T), dtype=torch.float32, device="cuda").reshape(-1)
    got = pk.patch_backward(pk.DeviceObservation(obs), [src], G, prec).cpu().numpy()
    err = np.max(np.abs(got[0] - g_ref[0])) / np.max(np.abs(g_ref[0]))
    print(f"64x300 {prec}: dir rel err {err:.2e}", flush=True)
    assert err <= GRAD_TOL


def _loss_and_grads(pk, fn, lm_s, f_s, T, dobs, srcs, prec, ws, d):
    """Forward (one batched call), loss and backward (one adjoint call) of
    the fitting loss at lm_s, with directions in the device array d."""
    lm = lm_s.detach().clone().requires_grad_(True)
    f = f_s.detach().clone().requires_grad_(True)
    out = fn.apply(lm, f, dobs, srcs, prec, ws, d)
    loss = ((out.double() - T.double()) ** 2).sum()
    loss.backward()
    return loss.detach(), lm.grad, f.grad


def test_captured_forward_backward_replays_new_directions(pk):
    """The forward (psf_patch_batched), the loss and the backward
    (psf_flux_backward, psf_patch_backward) of the fitting loss captured once
    into a HIP graph with the directions in a device source array; replays
    after writing new directions into the captured input give gradients
    bit-equal to eager calls at the same directions and within 1e-4 of the
    FP64 oracle's analytic gradient there."""
    prec = "split_bf16"
    obs, srcs, fluxes, targets = _config1_case()
    dobs = pk.DeviceObservation(obs)
    fn = pk.psf_patch_fn()
    ws = pk.Workspace()
    ws.get(pk.workspace_bytes(dobs, srcs, prec))
    _, d = pk.device_sources(srcs)
    T = torch.as_tensor(np.stack(targets), dtype=torch.float32, device="cuda")
    lm_s = torch.tensor([[s.l0, s.m0] for s in srcs], dtype=torch.float64, device="cuda")
    f_s = torch.tensor(fluxes, dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside capture, as torch asks
        for _ in range(2):
            _loss_and_grads(pk, fn, lm_s, f_s, T, dobs, srcs, prec, ws, d)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        L_g, glm_g, gf_g = _loss_and_grads(pk, fn, lm_s, f_s, T, dobs, srcs, prec, ws, d)
    rng = np.random.default_rng(17)
    for rep in range(3):
        new = np.array([[s.l0, s.m0] for s in srcs]) + rng.normal(0.0, 2 * ps.ARCSEC, (len(srcs), 2))
        lm_s.copy_(torch.as_tensor(new, dtype=torch.float64))
        g.replay()
        torch.cuda.synchronize()
        got_lm, got_f, got_L = glm_g.cpu().numpy().copy(), gf_g.double().cpu().numpy(), float(L_g)
        # eager calls at the same directions, on fresh device arrays
        _, d2 = pk.device_sources(srcs)
        L_e, glm_e, gf_e = _loss_and_grads(pk, fn, lm_s, f_s, T, dobs, srcs, prec, pk.Workspace(), d2)
        torch.cuda.synchronize()
        assert np.array_equal(got_lm, glm_e.cpu().numpy()), rep
        assert np.array_equal(got_f, gf_e.double().cpu().numpy()), rep
        assert got_L == float(L_e)
        moved = [s.with_direction(float(a), float(b)) for s, (a, b) in zip(srcs, new)]
        T64 = [t.astype(np.float64) for t in targets]
        L_ref, g_ref, gf_ref = orc.loss_grad_analytic(obs, moved, fluxes, T64)
        assert abs(got_L - L_ref) <= 1e-3 * L_ref
        for s in range(len(srcs)):
            err = np.max(np.abs(got_lm[s] - g_ref[s])) / np.max(np.abs(g_ref[s]))
            ferr = abs(got_f[s] - gf_ref[s]) / abs(gf_ref[s])
            print(f"replay {rep} src{s}: dir rel err {err:.2e}, flux rel err {ferr:.2e}", flush=True)
            assert err <= GRAD_TOL and ferr <= GRAD_TOL, (rep, s)


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_backward_small_column_steps(pk, prec):
    """Baselines of a few metres at a 0.05 arcsec cell on 257 x 257 patches:
    the column step of every phase factor is 1e-5 to 1e-4 rad, where the
    adjoint's column recurrence (a rounded 2 cos t over 8 columns, then
    complex jumps of 25 columns, over all nine k-steps of a row) is least
    accurate per element; against the FP64 analytic gradient."""
    obs = ps.tiny_random(51, n_ant=8, n_t=60, n_ch=4, nt=3, nc=2, radius_m=10.0, dt=60.0)
    cell = 0.05 * ps.ARCSEC
    srcs = [ps.Source.centred(0.003, -0.002, 257, cell), ps.Source.centred(-0.001, 0.004, 257, cell, nm=255)]
    g = np.random.default_rng(23)
    for src in srcs:
        T = orc.patch_factored(obs, src.with_direction(src.l0 + g.normal(0, 0.05 * ps.ARCSEC),
                                                       src.m0 + g.normal(0, 0.05 * ps.ARCSEC)))
        _, g_ref, _ = orc.loss_grad_analytic(obs, [src], [1.0], [T])
        G = torch.as_tensor(2.0 * (orc.patch_factored(obs, src) - T), dtype=torch.float32, device="cuda").reshape(-1)
        got = pk.patch_backward(pk.DeviceObservation(obs), [src], G, prec).cpu().numpy()
        err = np.max(np.abs(got[0] - g_ref[0])) / np.max(np.abs(g_ref[0]))
        print(f"small column steps {src.nl}x{src.nm} {prec}: dir rel err {err:.2e}", flush=True)
        assert err <= GRAD_TOL
