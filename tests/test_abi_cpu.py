"""The C-ABI library builds, loads and exports every declared symbol; host
validation rejects bad arguments before anything is launched (CPU only:
no call here reaches the device)."""
import ctypes
import os
import re

import pytest

import paper_2009_07010_amd as pk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psf.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(pk.LIB_PATH):
        from paper_2009_07010_amd import build
        build.build(verbose=False)
    return pk.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psf_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("psf_decorr", "psf_patch", "psf_patch_batched", "psf_patch_backward"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    for name in declared_functions():
        assert hasattr(L, name), name
        assert name in pk.EXPORTED, f"binding lacks {name}"


def test_strerror_and_version(L):
    for st in (0, -1, -2, -3, -4):
        assert L.psf_strerror(st)
    assert b"gfx950" in L.psf_version()


FAKE = 0x1000  # never dereferenced: every call below fails validation first


def fake_obs(**kw):
    o = pk.PsfObs(n_bl=3, n_t=10, n_ch=4, reserved=0, K=12, n_tb=6, uvw_m=FAKE, freq_hz=FAKE, bl_bin=FAKE,
                  bl_koff=FAKE, bl_tboff=FAKE, uvw_c_m=FAKE, W=FAKE)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def fake_src(**kw):
    s = pk.PsfSrc(l0=0.01, m0=0.02, l_first=0.0, m_first=0.0, dl=1e-5, dm=1e-5, nl=65, nm=65, out_off=0)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def status_of(fn, *args):
    st = fn(*args)
    return st, pk.lib().psf_last_error().decode()


@pytest.mark.parametrize("bad", [
    dict(uvw_m=None), dict(W=None), dict(n_t=0), dict(n_ch=-1), dict(K=2), dict(reserved=1),
    dict(K=10 ** 9),
])
def test_bad_observation_rejected(L, bad):
    o = fake_obs(**bad)
    srcs = (pk.PsfSrc * 1)(fake_src())
    out = ctypes.c_size_t(0)
    st, msg = status_of(L.psf_workspace_bytes, ctypes.byref(o), 1, srcs, 0, ctypes.byref(out))
    assert st == pk.PSF_EINVAL and msg


@pytest.mark.parametrize("bad", [dict(nl=0), dict(nm=5000), dict(l0=0.9, m0=0.9), dict(dl=float("nan")),
                                 dict(out_off=-1)])
def test_bad_source_rejected(L, bad):
    o = fake_obs()
    s = fake_src(**bad)
    st, msg = status_of(L.psf_patch, ctypes.byref(o), ctypes.byref(s), None, 0, FAKE, FAKE, 1 << 30, None)
    assert st == pk.PSF_EINVAL and msg


def test_bad_precision_and_null_output(L):
    o, s = fake_obs(), fake_src()
    st, _ = status_of(L.psf_patch, ctypes.byref(o), ctypes.byref(s), None, 7, FAKE, FAKE, 1 << 30, None)
    assert st == pk.PSF_EINVAL
    st, _ = status_of(L.psf_patch, ctypes.byref(o), ctypes.byref(s), None, 0, None, FAKE, 1 << 30, None)
    assert st == pk.PSF_EINVAL


def test_mixed_and_stochastic_precisions_accepted_and_next_value_rejected(L):
    # PSF_MIXED_FP16 and PSF_SR_FP16 pass validation; the next value is unknown
    o = fake_obs()
    srcs = (pk.PsfSrc * 1)(fake_src())
    for p in (pk.PSF_MIXED_FP16, pk.PSF_SR_FP16):
        need = ctypes.c_size_t(0)
        assert L.psf_workspace_bytes(ctypes.byref(o), 1, srcs, p, ctypes.byref(need)) == 0
        assert need.value > 12 * 40
    out = ctypes.c_size_t(0)
    st, msg = status_of(L.psf_workspace_bytes, ctypes.byref(o), 1, srcs, pk.PSF_SR_FP16 + 1, ctypes.byref(out))
    assert st == pk.PSF_EINVAL and "precision" in msg
    assert pk.PRECISIONS["mixed_fp16"] == pk.PSF_MIXED_FP16 == 4
    assert pk.PRECISIONS["sr_fp16"] == pk.PSF_SR_FP16 == 5


def test_workspace_too_small(L):
    o, s = fake_obs(), fake_src()
    srcs = (pk.PsfSrc * 1)(s)
    need = ctypes.c_size_t(0)
    assert L.psf_workspace_bytes(ctypes.byref(o), 1, srcs, 1, ctypes.byref(need)) == 0
    assert need.value > 12 * 40
    # the reported size covers every entry point; the records alone (40 B per
    # bin and source: u', v', two step factors, W D) already exceed 12 * 24 - 1 bytes
    st, msg = status_of(L.psf_patch, ctypes.byref(o), ctypes.byref(s), None, 1, FAKE, FAKE, 12 * 24 - 1, None)
    assert st == pk.PSF_EWORKSPACE and "workspace" in msg
    st, _ = status_of(L.psf_patch, ctypes.byref(o), ctypes.byref(s), None, 1, FAKE, None, need.value, None)
    assert st == pk.PSF_EWORKSPACE
    grad = FAKE
    st, msg = status_of(L.psf_patch_backward, ctypes.byref(o), 1, srcs, None, FAKE, 1, grad, FAKE,
                        12 * 24 - 1, None)
    assert st == pk.PSF_EWORKSPACE and "workspace" in msg


def test_backward_argument_errors(L):
    o, s = fake_obs(), fake_src()
    srcs = (pk.PsfSrc * 1)(s)
    st, _ = status_of(L.psf_patch_backward, ctypes.byref(o), 0, srcs, None, FAKE, 1, FAKE, FAKE, 1 << 30, None)
    assert st == pk.PSF_EINVAL
    st, _ = status_of(L.psf_patch_backward, ctypes.byref(o), 1, srcs, None, None, 1, FAKE, FAKE, 1 << 30, None)
    assert st == pk.PSF_EINVAL
    st, _ = status_of(L.psf_patch_backward, ctypes.byref(o), 1, srcs, None, FAKE, 9, FAKE, FAKE, 1 << 30, None)
    assert st == pk.PSF_EINVAL


def test_decorr_bad_direction(L):
    o = fake_obs()
    st, _ = status_of(L.psf_decorr, ctypes.byref(o), 0.8, 0.8, FAKE, None)
    assert st == pk.PSF_EINVAL
    st, _ = status_of(L.psf_decorr_sinc, ctypes.byref(o), 0.8, 0.8, FAKE, None)
    assert st == pk.PSF_EINVAL
    st, _ = status_of(L.psf_decorr_sinc, ctypes.byref(o), 0.01, 0.01, None, None)
    assert st == pk.PSF_EINVAL
    st, _ = status_of(L.psf_decorr, ctypes.byref(o), float("inf"), 0.0, FAKE, None)
    assert st == pk.PSF_EINVAL


@pytest.mark.parametrize("field", ["win_t", "win_c"])
def test_method1_rejects_windowed_observation(L, field):
    o = fake_obs(**{field: FAKE})
    st, msg = status_of(L.psf_decorr_sinc, ctypes.byref(o), 0.01, 0.01, FAKE, None)
    assert st == pk.PSF_EINVAL and "window" in msg


def test_obs_struct_layout_matches_header():
    """The ctypes mirror of psf_obs: 4 int32, 2 int64, 9 pointers."""
    assert ctypes.sizeof(pk.PsfObs) == 4 * 4 + 2 * 8 + 9 * 8
    assert pk.PsfObs.win_c.offset == ctypes.sizeof(pk.PsfObs) - 8


def test_binding_raises_on_error(L):
    with pytest.raises(pk.PsfError) as ei:
        pk.psf_decorr(fake_obs(n_t=0), 0.0, 0.0, FAKE, 0)
    assert ei.value.status == pk.PSF_EINVAL


def test_clean_argument_errors(L):
    o, g = fake_obs(), fake_src()
    n = ctypes.c_int32(0)
    ci = (ctypes.c_int32 * 4)()
    cj = (ctypes.c_int32 * 4)()
    ca = (ctypes.c_float * 4)()
    args = lambda res, iters, gain, thr, ws, wsb: (ctypes.byref(o), ctypes.byref(g), res, iters, gain, thr, 1, ci, cj,
                                                  ca, ctypes.byref(n), ws, wsb, None)
    st, _ = status_of(L.psf_clean_hogbom, *args(FAKE, 4, 0.0, 0.0, FAKE, 1 << 30))
    assert st == pk.PSF_EINVAL
    st, _ = status_of(L.psf_clean_hogbom, *args(FAKE, 4, 1.5, 0.0, FAKE, 1 << 30))
    assert st == pk.PSF_EINVAL
    st, _ = status_of(L.psf_clean_hogbom, *args(None, 4, 0.1, 0.0, FAKE, 1 << 30))
    assert st == pk.PSF_EINVAL
    st, _ = status_of(L.psf_clean_hogbom, *args(FAKE, -1, 0.1, 0.0, FAKE, 1 << 30))
    assert st == pk.PSF_EINVAL
    st, msg = status_of(L.psf_clean_hogbom, *args(FAKE, 4, 0.1, 0.0, FAKE, 16))
    assert st == pk.PSF_EWORKSPACE and "workspace" in msg
    need = ctypes.c_size_t(0)
    assert L.psf_clean_workspace_bytes(ctypes.byref(o), ctypes.byref(g), 1, ctypes.byref(need)) == 0
    assert need.value > 65 * 65 * 4


def test_clean_on_device_argument_errors(L):
    """psf_clean_hogbom_device validates like psf_clean_hogbom, on the host
    and before any launch (its component arrays are device pointers)."""
    o, g = fake_obs(), fake_src()
    args = lambda res, iters, gain, thr, comp, wsb: (ctypes.byref(o), ctypes.byref(g), res, iters, gain, thr, 1,
                                                    comp, comp, comp, FAKE, FAKE, wsb, None)
    for bad in (args(FAKE, 4, 0.0, 0.0, FAKE, 1 << 30), args(FAKE, 4, 1.5, 0.0, FAKE, 1 << 30),
                args(None, 4, 0.1, 0.0, FAKE, 1 << 30), args(FAKE, -1, 0.1, 0.0, FAKE, 1 << 30),
                args(FAKE, 4, 0.1, -1.0, FAKE, 1 << 30), args(FAKE, 4, 0.1, 0.0, None, 1 << 30)):
        st, _ = status_of(L.psf_clean_hogbom_device, *bad)
        assert st == pk.PSF_EINVAL
    st, msg = status_of(L.psf_clean_hogbom_device, *args(FAKE, 4, 0.1, 0.0, FAKE, 16))
    assert st == pk.PSF_EWORKSPACE and "workspace" in msg


def test_clean_method2_on_device_argument_errors(L):
    g = fake_src()
    args = lambda N, res, iters, gain, thr, nu, comp, wsb: (N, FAKE, ctypes.byref(g), res, iters, gain, thr, 30.0,
                                                           1e6, nu, comp, comp, comp, FAKE, FAKE, wsb, None)
    for bad in (args(100, FAKE, 4, 0.1, 0.0, 1.4e9, FAKE, 1 << 30), args(64, None, 4, 0.1, 0.0, 1.4e9, FAKE, 1 << 30),
                args(64, FAKE, -1, 0.1, 0.0, 1.4e9, FAKE, 1 << 30), args(64, FAKE, 4, 0.0, 0.0, 1.4e9, FAKE, 1 << 30),
                args(64, FAKE, 4, 0.1, 0.0, 0.0, FAKE, 1 << 30), args(64, FAKE, 4, 0.1, 0.0, 1.4e9, None, 1 << 30)):
        st, _ = status_of(L.psf_clean_hogbom_method2_device, *bad)
        assert st == pk.PSF_EINVAL
    st, msg = status_of(L.psf_clean_hogbom_method2_device, *args(64, FAKE, 4, 0.1, 0.0, 1.4e9, FAKE, 16))
    assert st == pk.PSF_EWORKSPACE and "workspace" in msg


def test_fullw_host_side_errors(L):
    o = fake_obs()
    n = ctypes.c_int32(0)
    outside = fake_src(l0=0.9, m0=0.0, l_first=0.9, dl=0.01, nl=20)      # far corner at l = 1.09
    st, msg = status_of(L.psf_patch_fullw, ctypes.byref(o), ctypes.byref(outside), 1, FAKE, ctypes.byref(n),
                        FAKE, 1 << 40, None)
    assert st == pk.PSF_EINVAL and "sky" in msg
    s = fake_src()
    st, _ = status_of(L.psf_patch_fullw, ctypes.byref(o), ctypes.byref(s), 1, None, ctypes.byref(n), FAKE,
                      1 << 40, None)
    assert st == pk.PSF_EINVAL
    st, _ = status_of(L.psf_patch_fullw, ctypes.byref(o), ctypes.byref(s), 1, FAKE, ctypes.byref(n), FAKE, 16,
                      None)
    assert st == pk.PSF_EWORKSPACE
    st, _ = status_of(L.psf_patch_fullw, ctypes.byref(o), ctypes.byref(s), 7, FAKE, ctypes.byref(n), FAKE,
                      1 << 40, None)
    assert st == pk.PSF_EINVAL


def test_method2_host_side_errors(L):
    o = fake_obs()
    out = ctypes.c_size_t(0)
    assert L.psf_method2_workspace_bytes(ctypes.byref(o), 100, 1, 1, ctypes.byref(out)) == pk.PSF_EINVAL
    assert L.psf_method2_workspace_bytes(ctypes.byref(o), 128, 1, 4, ctypes.byref(out)) == pk.PSF_OK
    assert out.value >= 4 * 128 * 128 * 8
    st, _ = status_of(L.psf_method2_spectrum, ctypes.byref(o), 128, 0.0, 1, FAKE, FAKE, 1 << 40, None)
    assert st == pk.PSF_EINVAL
    dirs = (ctypes.c_double * 4)(0.01, 0.0, 0.9, 0.9)
    st, msg = status_of(L.psf_method2_patch, 128, 1e-5, FAKE, 2, dirs, 20.0, 1e6, 1.4e9, FAKE, FAKE, 1 << 40, None)
    assert st == pk.PSF_EINVAL and "sky" in msg
    st, _ = status_of(L.psf_method2_patch, 128, 1e-5, FAKE, 1, dirs, -1.0, 1e6, 1.4e9, FAKE, FAKE, 1 << 40, None)
    assert st == pk.PSF_EINVAL
    st, _ = status_of(L.psf_method2_patch, 128, 1e-5, FAKE, 1, dirs, 20.0, 1e6, 1.4e9, FAKE, FAKE, 1024, None)
    assert st == pk.PSF_EWORKSPACE


def test_successful_call_clears_last_error(L):
    o = fake_obs()
    out = ctypes.c_size_t(0)
    assert L.psf_method2_workspace_bytes(ctypes.byref(o), 100, 1, 1, ctypes.byref(out)) == pk.PSF_EINVAL
    assert L.psf_last_error()
    assert L.psf_method2_workspace_bytes(ctypes.byref(o), 128, 1, 1, ctypes.byref(out)) == pk.PSF_OK
    assert L.psf_last_error() == b""


def test_method2_clean_host_side_errors(L):
    out = ctypes.c_size_t(0)
    sq = fake_src(dl=1e-5, dm=1e-5)
    assert L.psf_clean_method2_workspace_bytes(128, ctypes.byref(sq), ctypes.byref(out)) == pk.PSF_OK
    assert out.value >= 128 * 128 * 12
    rect = fake_src(dl=1e-5, dm=2e-5)
    assert L.psf_clean_method2_workspace_bytes(128, ctypes.byref(rect), ctypes.byref(out)) == pk.PSF_EINVAL
    assert L.psf_clean_method2_workspace_bytes(100, ctypes.byref(sq), ctypes.byref(out)) == pk.PSF_EINVAL
    n = ctypes.c_int32(0)
    st, _ = status_of(L.psf_clean_hogbom_method2, 128, FAKE, ctypes.byref(sq), FAKE, 5, 1.5, 0.0, 20.0, 1e6, 1.4e9,
                      FAKE, FAKE, FAKE, ctypes.byref(n), FAKE, 1 << 40, None)
    assert st == pk.PSF_EINVAL
    st, _ = status_of(L.psf_clean_hogbom_method2, 128, FAKE, ctypes.byref(sq), FAKE, 5, 0.5, 0.0, 20.0, 1e6, 1.4e9,
                      FAKE, FAKE, FAKE, ctypes.byref(n), FAKE, 64, None)
    assert st == pk.PSF_EWORKSPACE


def test_flux_entry_points_host_side_errors(L):
    assert L.psf_flux_scale(0, 10, FAKE, FAKE, FAKE, None) == pk.PSF_EINVAL
    assert L.psf_flux_scale(2, 0, FAKE, FAKE, FAKE, None) == pk.PSF_EINVAL
    assert L.psf_flux_scale(2, 10, None, FAKE, FAKE, None) == pk.PSF_EINVAL
    assert L.psf_flux_backward(2, 10, FAKE, FAKE, FAKE, FAKE, None, None) == pk.PSF_EINVAL
    assert L.psf_flux_backward(70000, 10, FAKE, FAKE, FAKE, FAKE, FAKE, None) == pk.PSF_EINVAL


def test_normalise_flag(L):
    """PSF_NORMALISE is accepted where the normalised PSF is produced (and by
    the workspace query, whose size it does not change) and rejected by the
    entry points that do not produce it, before anything is launched."""
    o, s = fake_obs(), fake_src()
    srcs = (pk.PsfSrc * 1)(s)
    a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.psf_workspace_bytes(ctypes.byref(o), 1, srcs, 1, ctypes.byref(a)) == 0
    assert L.psf_workspace_bytes(ctypes.byref(o), 1, srcs, 1 | pk.PSF_NORMALISE, ctypes.byref(b)) == 0
    assert a.value == b.value
    st, _ = status_of(L.psf_patch, ctypes.byref(o), ctypes.byref(s), None, 1 | pk.PSF_NORMALISE, FAKE, FAKE, 1, None)
    assert st == pk.PSF_EWORKSPACE  # the flag passed validation
    st, _ = status_of(L.psf_patch, ctypes.byref(o), ctypes.byref(s), None, 0x200 | 1, FAKE, FAKE, 1, None)
    assert st == pk.PSF_EINVAL
    st, msg = status_of(L.psf_patch_backward, ctypes.byref(o), 1, srcs, None, FAKE, 1 | pk.PSF_NORMALISE, FAKE,
                        FAKE, 1 << 40, None)
    assert st == pk.PSF_EINVAL and "PSF_NORMALISE" in msg
    n = ctypes.c_int32(0)
    st, msg = status_of(L.psf_patch_fullw, ctypes.byref(o), ctypes.byref(s), 1 | pk.PSF_NORMALISE, FAKE,
                        ctypes.byref(n), FAKE, 1 << 40, None)
    assert st == pk.PSF_EINVAL and "PSF_NORMALISE" in msg
