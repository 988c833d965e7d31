"""ctypes binding of liblyaf.so (the C ABI in include/lyaf.h).

Argument marshalling only: every step of the optical-depth path runs in the
HIP kernels of the library.  Torch supplies device memory and the current
stream.  If the library is missing or fails to load, every call raises.

Functions mirror the C entry points:
  tau(...)                         -> lyaf_tau
  normalise_mean_flux(...)         -> lyaf_normalise_mean_flux
  normalise_mean_flux_noalloc(...) -> lyaf_normalise_mean_flux_noalloc
  field_skewers(...)               -> lyaf_field_skewers
  flux_power_3d(...)               -> lyaf_flux_power_3d
  normalise_mean_flux_backward(...)-> lyaf_normalise_mean_flux_backward
  tau_backward(...)                -> lyaf_tau_backward
  status_read(...)                 -> lyaf_status_read
and ``TauFlux`` wraps the forward (tau, rescale, F) and the hand-written
adjoint as a torch.autograd.Function.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblyaf.so")

LYAF_OK, LYAF_EINVAL, LYAF_EDOMAIN, LYAF_ENOROOT = 0, -1, -2, -3
LYAF_ENOCONV, LYAF_EDEVICE, LYAF_ENOMEM = -4, -5, -6
STATUS_DOMAIN, STATUS_NOROOT, STATUS_NOCONV = 1, 2, 4
FLAG_PLAIN, FLAG_PER_SKEWER, FLAG_PERSISTENT = 1, 2, 4
NUM_SHAPES = 6
PLAN_AUTOTUNE, PLAN_NO_GRAPH = 1, 2


def FLAG_SHAPE(v: int) -> int:
    """Force windowed-kernel shape v (LYAF_FLAG_SHAPE)."""
    return (int(v) + 1) << 8


EXPORTED = ("lyaf_tau", "lyaf_normalise_mean_flux", "lyaf_normalise_mean_flux_backward",
            "lyaf_tau_backward", "lyaf_status_read", "lyaf_strerror", "lyaf_version",
            "lyaf_plan_create", "lyaf_plan_execute", "lyaf_plan_status", "lyaf_plan_describe",
            "lyaf_plan_destroy", "lyaf_instrument", "lyaf_instrument_backward",
            "lyaf_angstrom_to_kms", "lyaf_lya_lyb_path_kms", "lyaf_flux_pdf",
            "lyaf_flux_power", "lyaf_kernel_timing", "lyaf_kernel_timing_read",
            "lyaf_normalise_mean_flux_noalloc", "lyaf_field_skewers", "lyaf_flux_power_3d")


class InstrumentParams(ctypes.Structure):
    _fields_ = [("fwhm_kms", ctypes.c_double), ("bin_kms", ctypes.c_double),
                ("v_start_kms", ctypes.c_double), ("noise_sigma", ctypes.c_double),
                ("window_k", ctypes.c_double)]


class FieldParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("box", ctypes.c_double), ("amp", ctypes.c_double),
                ("k_F", ctypes.c_double), ("E_plus", ctypes.c_double), ("dk", ctypes.c_double),
                ("n_table", ctypes.c_int64)]


class Power3dParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("box", ctypes.c_double), ("mean_F", ctypes.c_double),
                ("p_noise", ctypes.c_double), ("n_bins", ctypes.c_int64)]


class LyafError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str = ""):
        super().__init__(f"{what}: {msg or code} (code {code})")
        self.code = code


class Skewers(ctypes.Structure):
    _fields_ = [("n_skewers", ctypes.c_int64),
                ("offsets", ctypes.POINTER(ctypes.c_int64)),
                ("delta", ctypes.c_void_p), ("vpec", ctypes.c_void_p),
                ("dv", ctypes.c_void_p), ("T0", ctypes.c_void_p),
                ("gamma", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("tau_ref", ctypes.c_double), ("delta_pivot", ctypes.c_double),
                ("window_k", ctypes.c_double), ("flags", ctypes.c_uint32)]


_lib = None
_lock = threading.Lock()


def library_path() -> str:
    return LIB_PATH


def load():
    """Load liblyaf.so; raises if it is missing (no fallback exists)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_1105_4747_amd/build.py "
                "(hipcc, gfx950); there is no CPU fallback")
        from . import build as _build
        if _build.built_hash(LIB_PATH) != _build.source_hash():
            raise RuntimeError(
                f"{LIB_PATH} was not built from the current sources (csrc/*.hip, *.h, "
                "include/lyaf.h): rebuild it with paper_1105_4747_amd/build.py")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        PS, PP = ctypes.POINTER(Skewers), ctypes.POINTER(Params)
        lib.lyaf_tau.argtypes = [PS, PP, vp, vp]
        lib.lyaf_tau.restype = i32
        lib.lyaf_normalise_mean_flux.argtypes = [i64, vp, vp, dbl, vp, vp]
        lib.lyaf_normalise_mean_flux.restype = i32
        lib.lyaf_normalise_mean_flux_noalloc.argtypes = [i64, vp, vp, dbl, vp, vp, vp]
        lib.lyaf_normalise_mean_flux_noalloc.restype = i32
        lib.lyaf_normalise_mean_flux_backward.argtypes = [i64, vp, vp, vp, vp, i32, vp, vp]
        lib.lyaf_normalise_mean_flux_backward.restype = i32
        lib.lyaf_tau_backward.argtypes = [PS, PP, vp, vp, vp, vp, vp, vp]
        lib.lyaf_tau_backward.restype = i32
        lib.lyaf_status_read.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32)]
        lib.lyaf_status_read.restype = i32
        lib.lyaf_strerror.argtypes = [i32]
        lib.lyaf_strerror.restype = ctypes.c_char_p
        lib.lyaf_version.argtypes = []
        lib.lyaf_version.restype = i32
        lib.lyaf_plan_create.argtypes = [PS, PP, dbl, vp, vp, vp, ctypes.c_uint32, vp,
                                         ctypes.POINTER(vp)]
        lib.lyaf_plan_create.restype = i32
        lib.lyaf_plan_execute.argtypes = [vp, vp]
        lib.lyaf_plan_execute.restype = i32
        lib.lyaf_plan_status.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_uint32)]
        lib.lyaf_plan_status.restype = i32
        lib.lyaf_plan_describe.argtypes = [vp, ctypes.c_char_p, i64]
        lib.lyaf_plan_describe.restype = i32
        lib.lyaf_plan_destroy.argtypes = [vp]
        lib.lyaf_plan_destroy.restype = i32
        pi64 = ctypes.POINTER(ctypes.c_int64)
        PI = ctypes.POINTER(InstrumentParams)
        lib.lyaf_instrument.argtypes = [i64, pi64, vp, vp, PI, pi64, vp, vp, vp]
        lib.lyaf_instrument.restype = i32
        lib.lyaf_instrument_backward.argtypes = [i64, pi64, vp, PI, pi64, vp, vp, vp]
        lib.lyaf_instrument_backward.restype = i32
        lib.lyaf_angstrom_to_kms.argtypes = [dbl, dbl]
        lib.lyaf_angstrom_to_kms.restype = dbl
        lib.lyaf_lya_lyb_path_kms.argtypes = [dbl]
        lib.lyaf_lya_lyb_path_kms.restype = dbl
        lib.lyaf_flux_pdf.argtypes = [i64, vp, vp, vp]
        lib.lyaf_flux_pdf.restype = i32
        lib.lyaf_flux_power.argtypes = [i64, pi64, vp, vp, dbl, vp, vp]
        lib.lyaf_flux_power.restype = i32
        pi32 = ctypes.POINTER(ctypes.c_int32)
        lib.lyaf_field_skewers.argtypes = [ctypes.POINTER(FieldParams), vp, vp, i64, pi32, pi32,
                                           vp, vp, vp]
        lib.lyaf_field_skewers.restype = i32
        lib.lyaf_flux_power_3d.argtypes = [ctypes.POINTER(Power3dParams), i64, vp, pi32, pi32,
                                           vp, vp, vp, vp, vp, vp]
        lib.lyaf_flux_power_3d.restype = i32
        lib.lyaf_kernel_timing.argtypes = [i32]
        lib.lyaf_kernel_timing.restype = i32
        lib.lyaf_kernel_timing_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(dbl), pi64]
        lib.lyaf_kernel_timing_read.restype = i32
        _lib = lib
        return lib


def strerror(code: int) -> str:
    return load().lyaf_strerror(int(code)).decode()


def _check(rc: int, what: str):
    if rc != LYAF_OK:
        raise LyafError(rc, what, strerror(rc))


def _ptr(t):
    """Device pointer of a torch tensor (or None -> NULL)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _host_offsets(offsets):
    """int64 host array of skewer offsets (numpy, list or CPU tensor)."""
    if hasattr(offsets, "detach"):
        offsets = offsets.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))


def make_skewers(delta, vpec, dv, T0, gamma, offsets):
    """Fill the C struct; the returned tuple keeps the host offsets alive."""
    off = _host_offsets(offsets)
    sk = Skewers(len(off) - 1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                 _ptr(delta), _ptr(vpec), _ptr(dv), _ptr(T0), _ptr(gamma))
    return sk, off


def make_params(tau_ref=1.0, delta_pivot=10.0, window_k=6.0, flags=0):
    return Params(float(tau_ref), float(delta_pivot), float(window_k), int(flags))


def tau(delta, vpec, dv, T0, gamma, offsets, out, tau_ref=1.0, delta_pivot=10.0,
        window_k=6.0, flags=0, stream=None):
    """lyaf_tau: raw optical depth into ``out`` (float32 device [P])."""
    sk, _off = make_skewers(delta, vpec, dv, T0, gamma, offsets)
    prm = make_params(tau_ref, delta_pivot, window_k, flags)
    _check(load().lyaf_tau(ctypes.byref(sk), ctypes.byref(prm), _ptr(out), _stream(stream)),
           "lyaf_tau")
    return out


def normalise_mean_flux(tau_inout, F_out, target_F, A_out, stream=None):
    """lyaf_normalise_mean_flux: tau_inout <- A tau, F_out <- exp(-A tau),
    A_out (float64 device scalar) <- A."""
    _check(load().lyaf_normalise_mean_flux(tau_inout.numel(), _ptr(tau_inout), _ptr(F_out),
                                           float(target_F), _ptr(A_out), _stream(stream)),
           "lyaf_normalise_mean_flux")


NORM_NOALLOC_SCRATCH_BYTES = 131840  # LYAF_NORM_NOALLOC_SCRATCH_BYTES


def normalise_mean_flux_noalloc(tau_inout, F_out, target_F, A_out, status=None, stream=None):
    """lyaf_normalise_mean_flux_noalloc: as normalise_mean_flux, with the
    library's scratch in a static device array (no allocation); LYAF_STATUS_*
    bits are OR'd into ``status`` (uint32/int32 device scalar) when given."""
    _check(load().lyaf_normalise_mean_flux_noalloc(
        tau_inout.numel(), _ptr(tau_inout), _ptr(F_out), float(target_F), _ptr(A_out),
        _ptr(status), _stream(stream)), "lyaf_normalise_mean_flux_noalloc")


def normalise_mean_flux_backward(tau_raw, A, grad_F, grad_tau_scaled, implicit_A, out,
                                 stream=None):
    _check(load().lyaf_normalise_mean_flux_backward(
        tau_raw.numel(), _ptr(tau_raw), _ptr(A), _ptr(grad_F), _ptr(grad_tau_scaled),
        int(bool(implicit_A)), _ptr(out), _stream(stream)),
        "lyaf_normalise_mean_flux_backward")


def tau_backward(delta, vpec, dv, T0, gamma, offsets, grad_tau_raw, grad_delta, grad_vpec,
                 grad_T0=None, grad_gamma=None, tau_ref=1.0, delta_pivot=10.0,
                 window_k=6.0, flags=0, stream=None):
    sk, _off = make_skewers(delta, vpec, dv, T0, gamma, offsets)
    prm = make_params(tau_ref, delta_pivot, window_k, flags)
    _check(load().lyaf_tau_backward(ctypes.byref(sk), ctypes.byref(prm), _ptr(grad_tau_raw),
                                    _ptr(grad_delta), _ptr(grad_vpec), _ptr(grad_T0),
                                    _ptr(grad_gamma), _stream(stream)),
           "lyaf_tau_backward")


def angstrom_to_kms(dlambda, z) -> float:
    """lyaf_angstrom_to_kms: velocity width of ``dlambda`` A at Lyman alpha at ``z``."""
    return float(load().lyaf_angstrom_to_kms(float(dlambda), float(z)))


def lya_lyb_path_kms(proximity_kms=3000.0) -> float:
    """lyaf_lya_lyb_path_kms: Lya-Lyb path length minus the proximity zone, km/s."""
    return float(load().lyaf_lya_lyb_path_kms(float(proximity_kms)))


def make_instrument_params(fwhm_kms, bin_kms, v_start_kms=0.0, noise_sigma=0.0, window_k=6.0):
    return InstrumentParams(float(fwhm_kms), float(bin_kms), float(v_start_kms),
                            float(noise_sigma), float(window_k))


def instrument(F, dv, offsets, out_offsets, F_obs, fwhm_kms, bin_kms, v_start_kms=0.0,
               noise=None, noise_sigma=0.0, window_k=6.0, stream=None):
    """lyaf_instrument: line-spread convolution, resampling and noise of each
    skewer's flux ``F`` (float32 device [P]) into ``F_obs`` (float32 device
    [P_out]); ``noise`` holds standard-normal draws [P_out] when
    ``noise_sigma > 0``."""
    off, oo = _host_offsets(offsets), _host_offsets(out_offsets)
    ip = make_instrument_params(fwhm_kms, bin_kms, v_start_kms, noise_sigma, window_k)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    _check(load().lyaf_instrument(len(off) - 1, off.ctypes.data_as(pi64), _ptr(dv), _ptr(F),
                                  ctypes.byref(ip), oo.ctypes.data_as(pi64), _ptr(noise),
                                  _ptr(F_obs), _stream(stream)),
           "lyaf_instrument")
    return F_obs


def instrument_backward(grad_obs, dv, offsets, out_offsets, grad_F, fwhm_kms, bin_kms,
                        v_start_kms=0.0, window_k=6.0, stream=None):
    """lyaf_instrument_backward: grad_F [P] <- J^T grad_obs [P_out]."""
    off, oo = _host_offsets(offsets), _host_offsets(out_offsets)
    ip = make_instrument_params(fwhm_kms, bin_kms, v_start_kms, 0.0, window_k)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    _check(load().lyaf_instrument_backward(len(off) - 1, off.ctypes.data_as(pi64), _ptr(dv),
                                           ctypes.byref(ip), oo.ctypes.data_as(pi64),
                                           _ptr(grad_obs), _ptr(grad_F), _stream(stream)),
           "lyaf_instrument_backward")
    return grad_F


PDF_SLOTS = 24  # lyaf_flux_pdf: 21 bins, below, above, NaN


def flux_pdf(F, counts, stream=None):
    """lyaf_flux_pdf: counts (int64 device [24]) of F (float32 device) in the 21
    flux-PDF bins, then below, above and NaN."""
    _check(load().lyaf_flux_pdf(F.numel(), _ptr(F), _ptr(counts), _stream(stream)),
           "lyaf_flux_pdf")
    return counts


def mode_offsets(offsets):
    """Offsets of lyaf_flux_power's output: skewer s holds N_s/2 + 1 modes."""
    n = np.diff(_host_offsets(offsets))
    return np.concatenate([[0], np.cumsum(n // 2 + 1)]).astype(np.int64)


def flux_power(F, dv, offsets, mean_F, out, stream=None):
    """lyaf_flux_power: per-skewer P(k_m), m = 0 .. N_s/2 (float32 device, laid
    out by mode_offsets)."""
    off = _host_offsets(offsets)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    _check(load().lyaf_flux_power(len(off) - 1, off.ctypes.data_as(pi64), _ptr(dv), _ptr(F),
                                  float(mean_F), _ptr(out), _stream(stream)),
           "lyaf_flux_power")
    return out


def field_skewers(modes, pk, sx, sy, delta_b, v_z, n, box, amp, k_F, E_plus, dk,
                  stream=None):
    """lyaf_field_skewers: delta_b and v_z (float32 device [S, n]) on the
    sight-lines (sx[s], sy[s]) of the field whose Gaussian half-spectrum is
    ``modes`` (complex64 device [n, n, n/2+1]) and power table ``pk`` (float64
    device, P at |k| = j dk); eqs. (1) and (3)."""
    import torch
    assert modes.dtype == torch.complex64 and pk.dtype == torch.float64
    x = np.ascontiguousarray(np.asarray(sx, dtype=np.int32))
    y = np.ascontiguousarray(np.asarray(sy, dtype=np.int32))
    if x.shape != y.shape:
        raise ValueError("sx and sy differ in length")
    fp = FieldParams(int(n), float(box), float(amp), float(k_F), float(E_plus), float(dk),
                     int(pk.numel()))
    pi32 = ctypes.POINTER(ctypes.c_int32)
    _check(load().lyaf_field_skewers(ctypes.byref(fp), _ptr(modes), _ptr(pk), len(x),
                                     x.ctypes.data_as(pi32), y.ctypes.data_as(pi32),
                                     _ptr(delta_b), _ptr(v_z), _stream(stream)),
           "lyaf_field_skewers")
    return delta_b, v_z


def flux_power_3d(F, mean_F, sx, sy, n, box, n_bins, counts, k_mean, p_true, p_box,
                  weights=None, p_noise=0.0, stream=None):
    """lyaf_flux_power_3d: the reconstruction of eq. (7) from the sight-lines
    F (float32 device [S * n]) at columns (sx, sy), averaged in spherical shells
    of the fundamental wavenumber; the four outputs are float64 device
    [n_bins]: mode counts, mean |k|, mean P_true, mean P_box."""
    x = np.ascontiguousarray(np.asarray(sx, dtype=np.int32))
    y = np.ascontiguousarray(np.asarray(sy, dtype=np.int32))
    if x.shape != y.shape:
        raise ValueError("sx and sy differ in length")
    pp = Power3dParams(int(n), float(box), float(mean_F), float(p_noise), int(n_bins))
    pi32 = ctypes.POINTER(ctypes.c_int32)
    _check(load().lyaf_flux_power_3d(ctypes.byref(pp), len(x), _ptr(F),
                                     x.ctypes.data_as(pi32), y.ctypes.data_as(pi32),
                                     _ptr(weights), _ptr(counts), _ptr(k_mean), _ptr(p_true),
                                     _ptr(p_box), _stream(stream)),
           "lyaf_flux_power_3d")
    return counts, k_mean, p_true, p_box


def status_read(stream=None) -> int:
    v = ctypes.c_uint32(0)
    _check(load().lyaf_status_read(_stream(stream), ctypes.byref(v)), "lyaf_status_read")
    return int(v.value)


def version() -> int:
    return int(load().lyaf_version())


def kernel_timing(enable: bool) -> None:
    """lyaf_kernel_timing: start (clearing earlier records) or stop recording
    HIP events around the library's kernel launches."""
    _check(load().lyaf_kernel_timing(1 if enable else 0), "lyaf_kernel_timing")


def kernel_timing_read(name: str):
    """lyaf_kernel_timing_read: (total ms, launches) recorded under ``name``
    since the last read of it; waits for those launches."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(load().lyaf_kernel_timing_read(name.encode(), ctypes.byref(ms), ctypes.byref(n)),
           "lyaf_kernel_timing_read")
    return float(ms.value), int(n.value)


class Plan:
    """lyaf_plan_*: the whole forward (tau, mean-flux rescale, F) bound to
    fixed device buffers, captured once as a hipGraph and replayed.

    ``tau_out`` receives tau' = A tau, ``F_out`` receives F, ``A_out`` (a
    float64 device scalar) receives A.  The tensors passed here must stay
    alive (and at the same address) for the life of the plan."""

    def __init__(self, delta, vpec, dv, T0, gamma, offsets, target_F, tau_out, F_out, A_out,
                 tau_ref=1.0, delta_pivot=10.0, window_k=6.0, autotune=False, graph=True,
                 stream=None):
        sk, off = make_skewers(delta, vpec, dv, T0, gamma, offsets)
        prm = make_params(tau_ref, delta_pivot, window_k, 0)
        flags = (PLAN_AUTOTUNE if autotune else 0) | (0 if graph else PLAN_NO_GRAPH)
        h = ctypes.c_void_p()
        self._keep = (delta, vpec, dv, T0, gamma, tau_out, F_out, A_out, off)
        _check(load().lyaf_plan_create(ctypes.byref(sk), ctypes.byref(prm), float(target_F),
                                       _ptr(tau_out), _ptr(F_out), _ptr(A_out), flags,
                                       _stream(stream), ctypes.byref(h)), "lyaf_plan_create")
        self._h = h

    def execute(self, stream=None):
        _check(load().lyaf_plan_execute(self._h, _stream(stream)), "lyaf_plan_execute")

    def status(self, stream=None) -> int:
        v = ctypes.c_uint32(0)
        _check(load().lyaf_plan_status(self._h, _stream(stream), ctypes.byref(v)),
               "lyaf_plan_status")
        return int(v.value)

    def describe(self) -> dict:
        import json
        n = load().lyaf_plan_describe(self._h, None, 0)
        if n < 0:
            _check(n, "lyaf_plan_describe")
        buf = ctypes.create_string_buffer(n + 1)
        load().lyaf_plan_describe(self._h, buf, n + 1)
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().lyaf_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
def _autograd():
    import torch

    class TauFlux(torch.autograd.Function):
        """(Delta, v, T0, gamma) -> (tau', F) with the mean-flux rescale.

        forward : lyaf_tau, then lyaf_normalise_mean_flux.
        backward: lyaf_normalise_mean_flux_backward (A implicit unless
                  ``implicit_A`` is False), then lyaf_tau_backward.
        T0 and gamma are per-skewer float32 tensors; their gradients come back
        per skewer (the library sums them in FP64)."""

        @staticmethod
        def forward(ctx, delta, vpec, T0, gamma, dv, offsets, target_F, tau_ref,
                    delta_pivot, window_k, implicit_A):
            delta, vpec = delta.contiguous(), vpec.contiguous()
            T0, gamma, dv = T0.contiguous(), gamma.contiguous(), dv.contiguous()
            P = delta.numel()
            raw = torch.empty(P, device=delta.device, dtype=torch.float32)
            tau(delta, vpec, dv, T0, gamma, offsets, raw, tau_ref, delta_pivot, window_k)
            ts = raw.clone()
            F = torch.empty_like(raw)
            A = torch.empty((), device=delta.device, dtype=torch.float64)
            normalise_mean_flux(ts, F, target_F, A)
            ctx.save_for_backward(delta, vpec, T0, gamma, dv, raw, A)
            ctx.cfg = (offsets, tau_ref, delta_pivot, window_k, implicit_A)
            ctx.mark_non_differentiable(A)
            return ts, F, A

        @staticmethod
        def backward(ctx, g_ts, g_F, g_A):
            delta, vpec, T0, gamma, dv, raw, A = ctx.saved_tensors
            offsets, tau_ref, delta_pivot, window_k, implicit_A = ctx.cfg
            g_raw = torch.empty_like(raw)
            normalise_mean_flux_backward(
                raw, A, None if g_F is None else g_F.contiguous().float(),
                None if g_ts is None else g_ts.contiguous().float(), implicit_A, g_raw)
            gd = torch.empty_like(delta)
            gv = torch.empty_like(vpec)
            gT = torch.empty(T0.numel(), device=T0.device, dtype=torch.float64)
            gg = torch.empty(gamma.numel(), device=gamma.device, dtype=torch.float64)
            tau_backward(delta, vpec, dv, T0, gamma, offsets, g_raw, gd, gv, gT, gg,
                         tau_ref, delta_pivot, window_k)
            return (gd, gv, gT.to(T0.dtype), gg.to(gamma.dtype), None, None, None, None,
                    None, None, None)

    class Instrument(torch.autograd.Function):
        """F -> mock observation (line-spread convolution, resampling, noise).

        forward : lyaf_instrument; backward: lyaf_instrument_backward."""

        @staticmethod
        def forward(ctx, F, dv, offsets, out_offsets, fwhm_kms, bin_kms, v_start_kms, noise,
                    noise_sigma, window_k):
            F, dv = F.contiguous(), dv.contiguous()
            n_out = int(_host_offsets(out_offsets)[-1])
            out = torch.empty(n_out, device=F.device, dtype=torch.float32)
            instrument(F, dv, offsets, out_offsets, out, fwhm_kms, bin_kms, v_start_kms,
                       None if noise is None else noise.contiguous(), noise_sigma, window_k)
            ctx.save_for_backward(dv)
            ctx.cfg = (F.numel(), offsets, out_offsets, fwhm_kms, bin_kms, v_start_kms, window_k)
            return out

        @staticmethod
        def backward(ctx, g):
            (dv,) = ctx.saved_tensors
            P, offsets, out_offsets, fwhm_kms, bin_kms, v_start_kms, window_k = ctx.cfg
            gF = torch.empty(P, device=dv.device, dtype=torch.float32)
            instrument_backward(g.contiguous().float(), dv, offsets, out_offsets, gF, fwhm_kms,
                                bin_kms, v_start_kms, window_k)
            return gF, None, None, None, None, None, None, None, None, None

    return TauFlux, Instrument


_TauFlux = None
_Instrument = None


def tau_flux(delta, vpec, T0, gamma, dv, offsets, target_F, tau_ref=1.0, delta_pivot=10.0,
             window_k=6.0, implicit_A=True):
    """Differentiable (tau', F, A) for torch tensors on the GPU."""
    global _TauFlux, _Instrument
    if _TauFlux is None:
        _TauFlux, _Instrument = _autograd()
    return _TauFlux.apply(delta, vpec, T0, gamma, dv, offsets, target_F, tau_ref,
                          delta_pivot, window_k, implicit_A)


def observe(F, dv, offsets, out_offsets, fwhm_kms, bin_kms, v_start_kms=0.0, noise=None,
            noise_sigma=0.0, window_k=6.0):
    """Differentiable mock observation of ``F`` (torch tensors on the GPU)."""
    global _TauFlux, _Instrument
    if _Instrument is None:
        _TauFlux, _Instrument = _autograd()
    return _Instrument.apply(F, dv, offsets, out_offsets, fwhm_kms, bin_kms, v_start_kms, noise,
                             noise_sigma, window_k)
