"""Position-dependent PSFs of averaged visibilities on AMD MI355X.

Thin Python binding over the C ABI of ``libpsfdecorr.so`` (see
``include/psf.h``): argument marshalling only.  Every step of the PSF
computation runs in the library's HIP kernels; PyTorch supplies device
memory and the stream.  There is no CPU fallback: if the library is not
built, importing a function that needs it raises.

Low-level names mirror the C ABI (``psf_decorr``, ``psf_patch``,
``psf_patch_batched``, ``psf_patch_backward``, ``psf_workspace_bytes``,
``psf_autotune``); ``DeviceObservation`` and the lower-case helpers below
wrap them for torch tensors.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsfdecorr.so")

PSF_FP32, PSF_SPLIT_BF16, PSF_SPLIT_FP16, PSF_PLAIN_BF16, PSF_MIXED_FP16, PSF_SR_FP16 = 0, 1, 2, 3, 4, 5
PSF_NORMALISE = 0x100
PRECISIONS = {"fp32": PSF_FP32, "split_bf16": PSF_SPLIT_BF16, "split_fp16": PSF_SPLIT_FP16, "mixed_fp16": PSF_MIXED_FP16,
              "sr_fp16": PSF_SR_FP16, "plain_bf16": PSF_PLAIN_BF16}
PSF_OK, PSF_EINVAL, PSF_EWORKSPACE, PSF_EDEVICE, PSF_EUNSUPPORTED = 0, -1, -2, -3, -4


class PsfError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


class PsfObs(ctypes.Structure):
    _fields_ = [("n_bl", ctypes.c_int32), ("n_t", ctypes.c_int32), ("n_ch", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("K", ctypes.c_int64), ("n_tb", ctypes.c_int64),
                ("uvw_m", ctypes.c_void_p), ("freq_hz", ctypes.c_void_p), ("bl_bin", ctypes.c_void_p),
                ("bl_koff", ctypes.c_void_p), ("bl_tboff", ctypes.c_void_p), ("uvw_c_m", ctypes.c_void_p),
                ("W", ctypes.c_void_p), ("win_t", ctypes.c_void_p), ("win_c", ctypes.c_void_p)]


class PsfSrc(ctypes.Structure):
    _fields_ = [("l0", ctypes.c_double), ("m0", ctypes.c_double), ("l_first", ctypes.c_double),
                ("m_first", ctypes.c_double), ("dl", ctypes.c_double), ("dm", ctypes.c_double),
                ("nl", ctypes.c_int32), ("nm", ctypes.c_int32), ("out_off", ctypes.c_int64)]


_P = ctypes.c_void_p
_SIGNATURES = {
    "psf_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.c_int32, ctypes.POINTER(PsfSrc),
                                           ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "psf_decorr": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.c_double, ctypes.c_double, _P, _P]),
    "psf_decorr_sinc": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.c_double, ctypes.c_double, _P, _P]),
    "psf_method2_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.c_int32, ctypes.c_int,
                                                   ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "psf_method2_spectrum": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.c_int32, ctypes.c_double, ctypes.c_int,
                                            _P, _P, ctypes.c_size_t, _P]),
    "psf_method2_patch": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, _P, ctypes.c_int32, _P,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, _P, _P,
                                         ctypes.c_size_t, _P]),
    "psf_patch_fullw": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.POINTER(PsfSrc), ctypes.c_int, _P,
                                       ctypes.POINTER(ctypes.c_int32), _P, ctypes.c_size_t, _P]),
    "psf_patch": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.POINTER(PsfSrc), _P, ctypes.c_int, _P, _P,
                                 ctypes.c_size_t, _P]),
    "psf_patch_noalloc": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.POINTER(PsfSrc), _P, ctypes.c_int, _P,
                                         _P]),
    "psf_patch_batched": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.c_int32, ctypes.POINTER(PsfSrc), _P,
                                         ctypes.c_int, ctypes.c_char_p, _P, _P, ctypes.c_size_t, _P]),
    "psf_patch_backward": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.c_int32, ctypes.POINTER(PsfSrc), _P,
                                          _P, ctypes.c_int, _P, _P, ctypes.c_size_t, _P]),
    "psf_autotune": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.c_int32, ctypes.POINTER(PsfSrc),
                                    ctypes.c_int, _P, ctypes.c_size_t, ctypes.c_char_p, ctypes.c_size_t, _P]),
    "psf_clean_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.POINTER(PsfSrc), ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "psf_clean_hogbom": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.POINTER(PsfSrc), _P, ctypes.c_int32,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int, _P, _P, _P,
                                        ctypes.POINTER(ctypes.c_int32), _P, ctypes.c_size_t, _P]),
    "psf_clean_hogbom_device": (ctypes.c_int, [ctypes.POINTER(PsfObs), ctypes.POINTER(PsfSrc), _P, ctypes.c_int32,
                                               ctypes.c_double, ctypes.c_double, ctypes.c_int, _P, _P, _P, _P, _P,
                                               ctypes.c_size_t, _P]),
    "psf_clean_method2_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(PsfSrc),
                                                         ctypes.POINTER(ctypes.c_size_t)]),
    "psf_clean_hogbom_method2": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.POINTER(PsfSrc), _P, ctypes.c_int32,
                                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, _P, _P, _P, ctypes.POINTER(ctypes.c_int32), _P,
                                                ctypes.c_size_t, _P]),
    "psf_clean_hogbom_method2_device": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.POINTER(PsfSrc), _P,
                                                       ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, _P, _P,
                                                       _P, _P, _P, ctypes.c_size_t, _P]),
    "psf_flux_scale": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, _P, _P, _P, _P]),
    "psf_flux_backward": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, _P, _P, _P, _P, _P, _P]),
    "psf_timing_enable": (ctypes.c_int, [ctypes.c_int]),
    "psf_timing_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "psf_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "psf_last_error": (ctypes.c_char_p, []),
    "psf_version": (ctypes.c_char_p, []),
}
EXPORTED = tuple(_SIGNATURES)

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              f"`python -m paper_2009_07010_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != PSF_OK:
        L = lib()
        raise PsfError(status, f"{L.psf_strerror(status).decode()}: {L.psf_last_error().decode()}")


def _prec(p) -> int:
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


def make_src(src, out_off: int = 0) -> PsfSrc:
    """PsfSrc from any object with l0, m0, l_first, m_first, dl, dm, nl, nm."""
    return PsfSrc(float(src.l0), float(src.m0), float(src.l_first), float(src.m_first), float(src.dl),
                  float(src.dm), int(src.nl), int(src.nm), int(out_off))


def src_array(srcs: Sequence) -> "ctypes.Array":
    arr = (PsfSrc * len(srcs))()
    off = 0
    for n, s in enumerate(srcs):
        arr[n] = make_src(s, off)
        off += int(s.nl) * int(s.nm)
    return arr


# ---------------------------------------------------------------- raw ABI
def psf_workspace_bytes(obs: PsfObs, h_srcs, prec) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().psf_workspace_bytes(ctypes.byref(obs), len(h_srcs), h_srcs, _prec(prec), ctypes.byref(out)))
    return int(out.value)


def psf_decorr(obs: PsfObs, l0: float, m0: float, D_ptr: int, stream: int) -> None:
    _check(lib().psf_decorr(ctypes.byref(obs), l0, m0, D_ptr, stream))


def psf_decorr_sinc(obs: PsfObs, l0: float, m0: float, D_ptr: int, stream: int) -> None:
    _check(lib().psf_decorr_sinc(ctypes.byref(obs), l0, m0, D_ptr, stream))


def psf_patch(obs: PsfObs, h_src: PsfSrc, D_ptr: Optional[int], prec, P_ptr: int, ws_ptr: int,
              ws_bytes: int, stream: int) -> None:
    _check(lib().psf_patch(ctypes.byref(obs), ctypes.byref(h_src), D_ptr, _prec(prec), P_ptr, ws_ptr, ws_bytes,
                           stream))


def psf_patch_fullw(obs: PsfObs, h_src: PsfSrc, prec, P_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> int:
    n = ctypes.c_int32(0)
    _check(lib().psf_patch_fullw(ctypes.byref(obs), ctypes.byref(h_src), _prec(prec), P_ptr, ctypes.byref(n),
                                 ws_ptr, ws_bytes, stream))
    return int(n.value)


def psf_patch_batched(obs: PsfObs, h_srcs, d_srcs_ptr: int, prec, tuning_json: Optional[bytes], P_ptr: int,
                      ws_ptr: int, ws_bytes: int, stream: int) -> None:
    _check(lib().psf_patch_batched(ctypes.byref(obs), len(h_srcs), h_srcs, d_srcs_ptr, _prec(prec), tuning_json,
                                   P_ptr, ws_ptr, ws_bytes, stream))


def psf_patch_backward(obs: PsfObs, h_srcs, d_srcs_ptr: int, G_ptr: int, prec, grad_ptr: int, ws_ptr: int,
                       ws_bytes: int, stream: int) -> None:
    _check(lib().psf_patch_backward(ctypes.byref(obs), len(h_srcs), h_srcs, d_srcs_ptr, G_ptr, _prec(prec),
                                    grad_ptr, ws_ptr, ws_bytes, stream))


def psf_autotune(obs: PsfObs, h_srcs, prec, ws_ptr: int, ws_bytes: int, stream: int, cap: int = 1 << 16) -> str:
    buf = ctypes.create_string_buffer(cap)
    _check(lib().psf_autotune(ctypes.byref(obs), len(h_srcs), h_srcs, _prec(prec), ws_ptr, ws_bytes, buf, cap,
                              stream))
    return buf.value.decode()


def psf_timing_enable(on: bool) -> None:
    _check(lib().psf_timing_enable(1 if on else 0))


def psf_timing_read():
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().psf_timing_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# ---------------------------------------------------------------- torch layer
def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class DeviceObservation:
    """An observation's arrays resident in device memory, plus the ABI struct.

    ``obs`` is any object with the attributes of ``psf_synth.Observation``
    (uvw_m, freq_hz, bl_bin, bl_koff, bl_tboff, uvw_c_m, W as numpy arrays;
    optional averaging windows win_t [n_bl, n_t] and win_c [n_bl, n_ch]).
    """

    def __init__(self, obs, device="cuda"):
        torch = _torch()
        t = lambda a, dt: torch.as_tensor(a, dtype=dt).contiguous().to(device)
        self.uvw_m = t(obs.uvw_m, torch.float64)
        self.freq_hz = t(obs.freq_hz, torch.float64)
        self.bl_bin = t(obs.bl_bin, torch.int32)
        self.bl_koff = t(obs.bl_koff, torch.int64)
        self.bl_tboff = t(obs.bl_tboff, torch.int64)
        self.uvw_c_m = t(obs.uvw_c_m, torch.float64)
        self.W = t(obs.W, torch.float32)
        wt, wc = getattr(obs, "win_t", None), getattr(obs, "win_c", None)
        self.win_t = None if wt is None else t(wt, torch.float32)
        self.win_c = None if wc is None else t(wc, torch.float32)
        if self.win_t is not None:
            assert tuple(self.win_t.shape) == tuple(obs.uvw_m.shape[:2]), "win_t must be [n_bl, n_t]"
        if self.win_c is not None:
            assert tuple(self.win_c.shape) == (obs.uvw_m.shape[0], len(obs.freq_hz)), "win_c must be [n_bl, n_ch]"
        self.n_bl, self.n_t = int(obs.uvw_m.shape[0]), int(obs.uvw_m.shape[1])
        self.n_ch = int(len(obs.freq_hz))
        self.K = int(obs.bl_koff[-1])
        self.n_tb = int(obs.bl_tboff[-1])
        self.device = device
        self.struct = PsfObs(self.n_bl, self.n_t, self.n_ch, 0, self.K, self.n_tb, self.uvw_m.data_ptr(),
                             self.freq_hz.data_ptr(), self.bl_bin.data_ptr(), self.bl_koff.data_ptr(),
                             self.bl_tboff.data_ptr(), self.uvw_c_m.data_ptr(), self.W.data_ptr(),
                             None if self.win_t is None else self.win_t.data_ptr(),
                             None if self.win_c is None else self.win_c.data_ptr())


class Workspace:
    """A growable device scratch buffer for the library's calls."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes: int):
        torch = _torch()
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.buf


def workspace_bytes(dobs: DeviceObservation, srcs: Sequence, prec="split_bf16") -> int:
    return psf_workspace_bytes(dobs.struct, src_array(srcs), prec)


def decorr(dobs: DeviceObservation, l0: float, m0: float, out=None):
    """D_k as a complex64 tensor [K]."""
    torch = _torch()
    D = torch.empty((dobs.K, 2), dtype=torch.float32, device=dobs.device) if out is None else out
    psf_decorr(dobs.struct, float(l0), float(m0), D.data_ptr(), _stream_handle())
    return torch.view_as_complex(D)


def decorr_sinc(dobs: DeviceObservation, l0: float, m0: float, out=None):
    """Method-1 (sinc) decorrelation factors as a complex64 tensor [K]
    (imaginary parts zero); pass as ``D`` to ``patch`` for the Method-1 PSF."""
    torch = _torch()
    D = torch.empty((dobs.K, 2), dtype=torch.float32, device=dobs.device) if out is None else out
    psf_decorr_sinc(dobs.struct, float(l0), float(m0), D.data_ptr(), _stream_handle())
    return torch.view_as_complex(D)


def patch(dobs: DeviceObservation, src, prec="split_bf16", D=None, out=None, workspace: Optional[Workspace] = None,
          normalise: bool = False):
    """The distorted PSF patch of one source, float32 [nl, nm]; with
    ``normalise`` divided by its value at the source, 2 Re sum W D."""
    torch = _torch()
    hs = make_src(src)
    arr = (PsfSrc * 1)(hs)
    need = psf_workspace_bytes(dobs.struct, arr, prec)
    ws = (workspace or Workspace(dobs.device)).get(need)
    P = torch.empty((int(src.nl), int(src.nm)), dtype=torch.float32, device=dobs.device) if out is None else out
    D_ptr = None
    if D is not None:
        Dr = torch.view_as_real(D) if D.is_complex() else D
        D_ptr = Dr.data_ptr()
    code = _prec(prec) | (PSF_NORMALISE if normalise else 0)
    psf_patch(dobs.struct, hs, D_ptr, code, P.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle())
    return P


def patch_noalloc(dobs: DeviceObservation, src, prec="split_bf16", D=None, out=None, normalise: bool = False):
    """``patch`` on the library's fixed scratch (``psf_patch_noalloc``): no
    workspace is allocated; raises PsfError (PSF_EWORKSPACE) when the patch
    needs more than that scratch."""
    torch = _torch()
    hs = make_src(src)
    P = torch.empty((int(src.nl), int(src.nm)), dtype=torch.float32, device=dobs.device) if out is None else out
    D_ptr = None
    if D is not None:
        D_ptr = (torch.view_as_real(D) if D.is_complex() else D).data_ptr()
    code = _prec(prec) | (PSF_NORMALISE if normalise else 0)
    _check(lib().psf_patch_noalloc(ctypes.byref(dobs.struct), ctypes.byref(hs), D_ptr, code, P.data_ptr(),
                                   _stream_handle()))
    return P


def patch_fullw(dobs: DeviceObservation, src, prec="split_bf16", out=None, workspace: Optional[Workspace] = None):
    """The patch with the exact w phase, float32 [nl, nm], and the number of
    contractions its expansion took."""
    torch = _torch()
    hs = make_src(src)
    need = psf_workspace_bytes(dobs.struct, (PsfSrc * 1)(hs), prec)
    ws = (workspace or Workspace(dobs.device)).get(need)
    P = torch.empty((int(src.nl), int(src.nm)), dtype=torch.float32, device=dobs.device) if out is None else out
    n = psf_patch_fullw(dobs.struct, hs, prec, P.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle())
    return P, n


def method2_spectrum(dobs: DeviceObservation, N: int, cell: float, prec="split_bf16",
                     workspace: Optional[Workspace] = None):
    """Method 2, once per observation and grid: the DFT of the effective PSF
    on the centred N x N grid, complex64 [N, N] in DFT order."""
    torch = _torch()
    need = ctypes.c_size_t(0)
    _check(lib().psf_method2_workspace_bytes(ctypes.byref(dobs.struct), int(N), _prec(prec), 1, ctypes.byref(need)))
    ws = (workspace or Workspace(dobs.device)).get(need.value)
    S = torch.empty((int(N), int(N), 2), dtype=torch.float32, device=dobs.device)
    _check(lib().psf_method2_spectrum(ctypes.byref(dobs.struct), int(N), float(cell), _prec(prec), S.data_ptr(),
                                      ws.data_ptr(), ws.numel(), _stream_handle()))
    return torch.view_as_complex(S)


def method2_patches(S, cell: float, dirs, dt_bin: float, dnu_bin: float, nu: float, out=None,
                    workspace: Optional[Workspace] = None):
    """Method 2 per source: float32 [n_src, N, N] on the centred grid of
    offsets from each source; ``dirs`` is a sequence of (l0, m0)."""
    torch = _torch()
    N = int(S.shape[0])
    h = (ctypes.c_double * (2 * len(dirs)))(*[float(v) for d in dirs for v in d])
    ws = (workspace or Workspace(S.device)).get(min(len(dirs), 16) * N * N * 8)
    P = torch.empty((len(dirs), N, N), dtype=torch.float32, device=S.device) if out is None else out
    Sr = torch.view_as_real(S) if S.is_complex() else S
    _check(lib().psf_method2_patch(N, float(cell), Sr.data_ptr(), len(dirs), h, float(dt_bin), float(dnu_bin),
                                   float(nu), P.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle()))
    return P


def patch_backward(dobs: DeviceObservation, srcs: Sequence, G_all, prec="split_bf16",
                   workspace: Optional[Workspace] = None, d_srcs=None, out=None):
    """dLoss/d(l0, m0) [n_src, 2] float64 on the device, from G_all = dLoss/dP
    (float32, each source's [nl, nm] block concatenated in order).  With
    ``d_srcs`` (from ``device_sources``) the directions and grids are read
    from that device array at run time, not from ``srcs``."""
    torch = _torch()
    arr = src_array(srcs)
    need = psf_workspace_bytes(dobs.struct, arr, prec)
    ws = (workspace or Workspace(dobs.device)).get(need)
    total = sum(int(s.nl) * int(s.nm) for s in srcs)
    G = G_all.to(device=dobs.device, dtype=torch.float32).contiguous()
    if G.numel() != total:
        raise ValueError(f"G_all has {G.numel()} elements, the patches {total}")
    grad = torch.empty((len(srcs), 2), dtype=torch.float64, device=dobs.device) if out is None else out
    psf_patch_backward(dobs.struct, arr, None if d_srcs is None else d_srcs.data_ptr(), G.data_ptr(), prec,
                       grad.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle())
    return grad


def _psf_patch_fn():
    torch = _torch()

    class PsfPatchFn(torch.autograd.Function):
        """flux_s * P_s(l0_s, m0_s) for every source, [n_src, nl, nm] float32.

        ``lm0`` float64 [n_src, 2] on the observation's device, ``flux``
        [n_src]; ``grids`` gives each source's fixed pixel grid (l_first,
        m_first, dl, dm, nl, nm, all patches the same size).  ``lm0`` is
        written into the device source array ``d_srcs`` (from
        ``device_sources(grids)``; made here when not given, which copies
        from the host and so cannot be captured), then one batched forward
        call (``psf_patch_batched``) and one flux scaling run; the backward
        is one ``psf_flux_backward`` and one ``psf_patch_backward`` reading
        the same device array.  Nothing is read back to the host, so a
        forward and backward with a given ``d_srcs`` and ``workspace`` can be
        captured into a graph and replayed for new ``lm0``.
        """

        @staticmethod
        def forward(ctx, lm0, flux, dobs, grids, prec="split_bf16", workspace=None, d_srcs=None):
            shapes = {(int(g.nl), int(g.nm)) for g in grids}
            if len(shapes) != 1 or tuple(lm0.shape) != (len(grids), 2) or tuple(flux.shape) != (len(grids),):
                raise ValueError("need lm0 [n_src, 2], flux [n_src] and equal patch sizes")
            nl, nm = shapes.pop()
            n = len(grids)
            if d_srcs is None:
                d_srcs = device_sources(grids, dobs.device)[1]
            set_directions(d_srcs, lm0.detach().to(dtype=torch.float64))
            ws = workspace or Workspace(dobs.device)
            P = patch_batched(dobs, grids, prec=prec, workspace=ws, d_srcs=d_srcs).view(n, nl, nm)
            f = flux.detach().to(device=dobs.device, dtype=torch.float32).contiguous()
            out = torch.empty_like(P)
            _check(lib().psf_flux_scale(n, nl * nm, f.data_ptr(), P.data_ptr(), out.data_ptr(), _stream_handle()))
            ctx.save_for_backward(P, f)
            ctx.grids, ctx.dobs, ctx.prec, ctx.ws, ctx.d_srcs = grids, dobs, prec, ws, d_srcs
            ctx.lm_device, ctx.flux_device, ctx.flux_dtype = lm0.device, flux.device, flux.dtype
            return out

        @staticmethod
        def backward(ctx, grad_out):
            P, f = ctx.saved_tensors
            n, nl, nm = P.shape
            go = grad_out.to(device=P.device, dtype=torch.float32).contiguous()
            G = torch.empty(n * nl * nm, dtype=torch.float32, device=P.device)
            gflux = torch.empty(n, dtype=torch.float64, device=P.device)
            _check(lib().psf_flux_backward(n, nl * nm, f.data_ptr(), P.data_ptr(), go.data_ptr(), G.data_ptr(),
                                           gflux.data_ptr(), _stream_handle()))
            grad_flux = gflux.to(device=ctx.flux_device, dtype=ctx.flux_dtype)
            grad_lm = patch_backward(ctx.dobs, ctx.grids, G, ctx.prec, ctx.ws, d_srcs=ctx.d_srcs).to(ctx.lm_device)
            return grad_lm, grad_flux, None, None, None, None, None

    return PsfPatchFn


_PSF_PATCH_FN = None


def psf_patch_fn():
    """The torch.autograd.Function over the forward patch and its adjoint."""
    global _PSF_PATCH_FN
    if _PSF_PATCH_FN is None:
        _PSF_PATCH_FN = _psf_patch_fn()
    return _PSF_PATCH_FN


def device_sources(srcs: Sequence, device="cuda"):
    """(host PsfSrc array, device copy of it as a uint8 tensor).  The device
    copy is what the batched call reads directions and grids from at run
    time; write new directions into it (``set_directions``) to replay a
    captured graph for other sources."""
    torch = _torch()
    h = src_array(srcs)
    raw = bytes(memoryview(h).cast("B"))
    d = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
    return h, d


def set_directions(d_srcs, lm0) -> None:
    """Overwrite (l0, m0) of every source in a device source array with the
    rows of ``lm0`` (float64 [n_src, 2], same device); grids stay.  A
    device-to-device copy on the current stream (capturable)."""
    torch = _torch()
    n = lm0.shape[0]
    rec = ctypes.sizeof(PsfSrc) // 8
    view = d_srcs.view(torch.float64).view(n, rec)
    view[:, 0:2].copy_(lm0)


def patch_batched(dobs: DeviceObservation, srcs: Sequence, prec="split_bf16", tuning: Optional[str] = None,
                  out=None, workspace: Optional[Workspace] = None, d_srcs=None, normalise: bool = False):
    """Every source's patch in one call, concatenated float32 [sum nl*nm] in
    source order (``split_patches`` cuts it).  ``d_srcs`` (from
    ``device_sources``) may be passed to reuse a device source array;
    ``normalise`` divides each patch by its value at its source."""
    torch = _torch()
    h, d = device_sources(srcs, dobs.device) if d_srcs is None else (src_array(srcs), d_srcs)
    need = psf_workspace_bytes(dobs.struct, h, prec)
    ws = (workspace or Workspace(dobs.device)).get(need)
    total = sum(int(s.nl) * int(s.nm) for s in srcs)
    P = torch.empty(total, dtype=torch.float32, device=dobs.device) if out is None else out
    code = _prec(prec) | (PSF_NORMALISE if normalise else 0)
    psf_patch_batched(dobs.struct, h, d.data_ptr(), code, None if tuning is None else tuning.encode(),
                      P.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle())
    return P


def split_patches(P_all, srcs: Sequence):
    """The per-source [nl, nm] views of a concatenated patch array."""
    out, off = [], 0
    for s in srcs:
        n = int(s.nl) * int(s.nm)
        out.append(P_all[off:off + n].view(int(s.nl), int(s.nm)))
        off += n
    return out


def autotune(dobs: DeviceObservation, srcs: Sequence, prec="split_bf16", workspace: Optional[Workspace] = None) -> str:
    """Times candidate launch shapes per tile family on these sources and
    returns the JSON tuning table for ``patch_batched``."""
    h = src_array(srcs)
    need = psf_workspace_bytes(dobs.struct, h, prec)
    ws = (workspace or Workspace(dobs.device)).get(need)
    return psf_autotune(dobs.struct, h, prec, ws.data_ptr(), ws.numel(), _stream_handle())


def clean_hogbom(dobs: DeviceObservation, grid, dirty, max_iter: int, gain: float = 0.1, threshold: float = 0.0,
                 prec="split_bf16", workspace: Optional[Workspace] = None):
    """Hogbom CLEAN with the distorted PSF at every peak (``psf_clean_hogbom``).
    ``dirty`` is a float32 [nl, nm] image on the grid of ``grid``; returns
    (residual tensor, list of (i, j, amplitude))."""
    torch = _torch()
    h = make_src(grid)
    need = ctypes.c_size_t(0)
    _check(lib().psf_clean_workspace_bytes(ctypes.byref(dobs.struct), ctypes.byref(h), _prec(prec),
                                           ctypes.byref(need)))
    ws = (workspace or Workspace(dobs.device)).get(need.value)
    res = dirty.to(device=dobs.device, dtype=torch.float32).contiguous().clone()
    ci = (ctypes.c_int32 * max(1, max_iter))()
    cj = (ctypes.c_int32 * max(1, max_iter))()
    ca = (ctypes.c_float * max(1, max_iter))()
    n = ctypes.c_int32(0)
    _check(lib().psf_clean_hogbom(ctypes.byref(dobs.struct), ctypes.byref(h), res.data_ptr(), int(max_iter),
                                  float(gain), float(threshold), _prec(prec), ci, cj, ca, ctypes.byref(n),
                                  ws.data_ptr(), ws.numel(), _stream_handle()))
    return res, [(ci[k], cj[k], ca[k]) for k in range(n.value)]


def clean_hogbom_device(dobs: DeviceObservation, grid, residual, n_iter: int, gain: float = 0.1,
                        threshold: float = 0.0, prec="split_bf16", workspace: Optional[Workspace] = None,
                        comps=None):
    """Hogbom CLEAN kept on the device (``psf_clean_hogbom_device``): exactly
    ``n_iter`` cycles on ``residual`` (float32 [nl, nm] on the GPU, updated in
    place), no host synchronisation, so the call can be captured into a
    graph.  Returns (comp_i int32 [n_iter], comp_j, comp_amp float32
    [n_iter], n_comp int32 [1]), all device tensors (``comps`` may pass them
    in to be reused); the first n_comp entries are the components."""
    torch = _torch()
    h = make_src(grid)
    need = ctypes.c_size_t(0)
    _check(lib().psf_clean_workspace_bytes(ctypes.byref(dobs.struct), ctypes.byref(h), _prec(prec),
                                           ctypes.byref(need)))
    ws = (workspace or Workspace(dobs.device)).get(need.value)
    if comps is None:
        m = max(1, int(n_iter))
        comps = (torch.empty(m, dtype=torch.int32, device=dobs.device),
                 torch.empty(m, dtype=torch.int32, device=dobs.device),
                 torch.empty(m, dtype=torch.float32, device=dobs.device),
                 torch.empty(1, dtype=torch.int32, device=dobs.device))
    ci, cj, ca, n = comps
    _check(lib().psf_clean_hogbom_device(ctypes.byref(dobs.struct), ctypes.byref(h), residual.data_ptr(),
                                         int(n_iter), float(gain), float(threshold), _prec(prec), ci.data_ptr(),
                                         cj.data_ptr(), ca.data_ptr(), n.data_ptr(), ws.data_ptr(), ws.numel(),
                                         _stream_handle()))
    return comps


def clean_hogbom_method2(S, grid, dirty, max_iter: int, dt_bin: float, dnu_bin: float, nu: float,
                         gain: float = 0.1, threshold: float = 0.0, workspace: Optional[Workspace] = None):
    """Hogbom CLEAN with the Method-2 PSF at every peak
    (``psf_clean_hogbom_method2``); ``S`` from ``method2_spectrum`` at the
    image's cell.  Returns (residual tensor, list of (i, j, amplitude))."""
    torch = _torch()
    N = int(S.shape[0])
    h = make_src(grid)
    need = ctypes.c_size_t(0)
    _check(lib().psf_clean_method2_workspace_bytes(N, ctypes.byref(h), ctypes.byref(need)))
    ws = (workspace or Workspace(S.device)).get(need.value)
    res = dirty.to(device=S.device, dtype=torch.float32).contiguous().clone()
    Sr = torch.view_as_real(S) if S.is_complex() else S
    ci = (ctypes.c_int32 * max(1, max_iter))()
    cj = (ctypes.c_int32 * max(1, max_iter))()
    ca = (ctypes.c_float * max(1, max_iter))()
    n = ctypes.c_int32(0)
    _check(lib().psf_clean_hogbom_method2(N, Sr.data_ptr(), ctypes.byref(h), res.data_ptr(), int(max_iter),
                                          float(gain), float(threshold), float(dt_bin), float(dnu_bin), float(nu),
                                          ci, cj, ca, ctypes.byref(n), ws.data_ptr(), ws.numel(),
                                          _stream_handle()))
    return res, [(ci[k], cj[k], ca[k]) for k in range(n.value)]

def clean_hogbom_method2_device(S, grid, residual, n_iter: int, dt_bin: float, dnu_bin: float, nu: float,
                                gain: float = 0.1, threshold: float = 0.0, workspace: Optional[Workspace] = None,
                                comps=None):
    """Hogbom CLEAN with Method-2 PSFs kept on the device
    (``psf_clean_hogbom_method2_device``): exactly ``n_iter`` cycles on
    ``residual`` (float32 [nl, nm] on the GPU, updated in place), no host
    synchronisation.  Returns (comp_i, comp_j, comp_amp, n_comp) device
    tensors as ``clean_hogbom_device`` does."""
    torch = _torch()
    N = int(S.shape[0])
    h = make_src(grid)
    need = ctypes.c_size_t(0)
    _check(lib().psf_clean_method2_workspace_bytes(N, ctypes.byref(h), ctypes.byref(need)))
    ws = (workspace or Workspace(S.device)).get(need.value)
    if comps is None:
        m = max(1, int(n_iter))
        comps = (torch.empty(m, dtype=torch.int32, device=S.device),
                 torch.empty(m, dtype=torch.int32, device=S.device),
                 torch.empty(m, dtype=torch.float32, device=S.device),
                 torch.empty(1, dtype=torch.int32, device=S.device))
    ci, cj, ca, n = comps
    Sr = torch.view_as_real(S) if S.is_complex() else S
    _check(lib().psf_clean_hogbom_method2_device(N, Sr.data_ptr(), ctypes.byref(h), residual.data_ptr(),
                                                 int(n_iter), float(gain), float(threshold), float(dt_bin),
                                                 float(dnu_bin), float(nu), ci.data_ptr(), cj.data_ptr(),
                                                 ca.data_ptr(), n.data_ptr(), ws.data_ptr(), ws.numel(),
                                                 _stream_handle()))
    return comps

