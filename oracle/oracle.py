"""FP64 CPU oracle for the Lyman-alpha optical-depth path -- test infrastructure.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product library never does, and this
module imports nothing from the product package.

It is a thin ctypes wrapper over ``lyaf_oracle.c`` (plain C, IEEE double,
OpenMP over skewers), which follows Greig, Bolton & Wyithe (2011), Section 2.3:
eq. (4) (photo-ionisation equilibrium n_HI), eq. (5) with its pivot (power-law
temperature-density relation), eq. (6) (optical-depth sum over thermally
broadened Gaussian profiles) and the mean-flux normalisation paragraph that
closes Section 2.3.  The C file's header states every formula.

Parity status of each function (what pins it is listed in the tests):
  tau (full sum)          pinned: Gunn-Peterson closed form (Jacobi theta),
                          isolated-line Gaussian, equivalent width with the
                          Poisson-summation correction, pivot closed form,
                          shift / reflection / bulk-velocity equivariance,
                          40-digit brute force over the full image lattice.
  tau (windowed, k >= 8)  pinned against the full sum.
  tau_at (chosen pixels)  the full sum at chosen pixels of one skewer; pinned
                          bitwise against tau (full sum) on a ragged batch.
  mean_flux_A             pinned: uniform-tau closed form, two-level closed form,
                          scipy brentq, the printed <F> = 0.72 <-> tau_eff = 0.329.
  tau_grad, normalise_backward
                          pinned: central finite differences of the forward,
                          closed forms for L = sum tau.
  instrument              (``lyaf_instrument_oracle.c``: Gaussian line-spread
                          convolution, resampling onto coarser bins, noise;
                          Sections 3.1, 3.2 and 4) pinned: circular convolution
                          by numpy's FFT, Gaussian-through-Gaussian closed form
                          (widths add in quadrature), flat spectrum unchanged,
                          block means for aligned integer bins, exact
                          integration of the piecewise-constant spectrum by
                          numpy interpolation of its cumulative integral, flux
                          conservation, shift equivariance, the paper's printed
                          3.63 A ~ 224 km/s pair.
  instrument_backward     pinned: dot-product identity with the forward (a
                          linear map), central finite differences.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lyaf_oracle.c")
_SRC_INS = os.path.join(_HERE, "lyaf_instrument_oracle.c")
_LIB = os.path.join(_HERE, "liblyaf_oracle.so")
_lock = threading.Lock()
_lib = None

ORC_OK, ORC_EINVAL, ORC_EDOMAIN, ORC_ENOROOT, ORC_ENOCONV = 0, -1, -2, -3, -4


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", "-D_DEFAULT_SOURCE",
           "-o", _LIB + ".tmp", _SRC, _SRC_INS, "-lm"]
    if force or not os.path.exists(_LIB):
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        stale = (not os.path.exists(_LIB)
                 or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                 os.path.getmtime(_SRC_INS)))
        if stale:
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64, dbl, i32 = ctypes.c_int64, ctypes.c_double, ctypes.c_int
        pd = ctypes.POINTER(ctypes.c_double)
        pi64 = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_tau.argtypes = [i64, pi64, pd, pd, pd, pd, pd, dbl, dbl, dbl, pd]
        lib.oracle_tau.restype = i32
        lib.oracle_tau_at.argtypes = [i64, pi64, pd, pd, pd, pd, pd, dbl, dbl, i64, pi64, i64,
                                      pd]
        lib.oracle_tau_at.restype = i32
        lib.oracle_mean_flux_A.argtypes = [i64, pd, dbl, pd, ctypes.POINTER(i32)]
        lib.oracle_mean_flux_A.restype = i32
        lib.oracle_finalise.argtypes = [i64, pd, dbl, pd, pd]
        lib.oracle_finalise.restype = None
        lib.oracle_tau_grad.argtypes = [i64, pi64, pd, pd, pd, pd, pd, dbl, dbl,
                                        pd, pd, pd, pd, pd]
        lib.oracle_tau_grad.restype = i32
        lib.oracle_normalise_backward.argtypes = [i64, pd, dbl, pd, pd, i32, pd]
        lib.oracle_normalise_backward.restype = i32
        lib.oracle_source_params.argtypes = [dbl] * 6 + [pd] * 4
        lib.oracle_source_params.restype = None
        lib.oracle_doppler_b.argtypes = [dbl]
        lib.oracle_doppler_b.restype = dbl
        lib.oracle_min_image.argtypes = [dbl, dbl]
        lib.oracle_min_image.restype = dbl
        lib.oracle_instrument.argtypes = [i64, pi64, pd, pd, dbl, dbl, dbl, pi64, pd, dbl, pd]
        lib.oracle_instrument.restype = i32
        lib.oracle_instrument_backward.argtypes = [i64, pi64, pd, dbl, dbl, dbl, pi64, pd, pd]
        lib.oracle_instrument_backward.restype = i32
        for name in ("oracle_angstrom_to_kms",):
            getattr(lib, name).argtypes = [dbl, dbl]
            getattr(lib, name).restype = dbl
        for name in ("oracle_lya_lyb_path_kms", "oracle_lsf_b"):
            getattr(lib, name).argtypes = [dbl]
            getattr(lib, name).restype = dbl
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = i32
        _lib = lib
        return lib


def _d(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _offsets(n_skewers, n_pix, offsets):
    if offsets is None:
        if n_skewers == 0:
            return np.zeros(1, np.int64)
        assert n_pix % n_skewers == 0
        return np.arange(n_skewers + 1, dtype=np.int64) * (n_pix // n_skewers)
    return np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))


def _per_skewer(x, S):
    a = _d(x)
    if a.ndim == 0:
        a = np.full(S, float(a))
    return np.ascontiguousarray(a)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def doppler_b(T: float) -> float:
    """b = sqrt(2 k_B T / m_H) in km/s."""
    return float(_load().oracle_doppler_b(float(T)))


def min_image(d: float, V: float) -> float:
    return float(_load().oracle_min_image(float(d), float(V)))


def source_params(delta, dv, T0, gamma, tau_ref=1.0, delta_pivot=10.0):
    """(D, T, b, w) of one source pixel, eqs. (4)-(5)."""
    out = [ctypes.c_double() for _ in range(4)]
    _load().oracle_source_params(float(delta), float(dv), float(T0),
                                 float(gamma), float(tau_ref),
                                 float(delta_pivot),
                                 *[ctypes.byref(o) for o in out])
    return tuple(o.value for o in out)


def tau(delta, vpec, dv, T0, gamma, offsets=None, n_skewers=None,
        tau_ref=1.0, delta_pivot=10.0, window_k=0.0):
    """Raw optical depth of eq. (6) for every pixel (float64 [P]).

    ``delta``/``vpec`` are flat [P] arrays, skewer-major.  ``offsets`` [S+1]
    (host int64) delimits skewers; if None, ``n_skewers`` equal skewers.
    ``dv``, ``T0``, ``gamma`` are scalars or per-skewer arrays."""
    delta, vpec = _d(delta).ravel(), _d(vpec).ravel()
    P = delta.size
    if offsets is None and n_skewers is None:
        n_skewers = 1
    S = (len(offsets) - 1) if offsets is not None else int(n_skewers)
    off = _offsets(S, P, offsets)
    dv_, T0_, g_ = _per_skewer(dv, S), _per_skewer(T0, S), _per_skewer(gamma, S)
    out = np.empty(P, np.float64)
    rc = _load().oracle_tau(S, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            _p(delta), _p(vpec), _p(dv_), _p(T0_), _p(g_),
                            float(tau_ref), float(delta_pivot), float(window_k),
                            _p(out))
    if rc:
        raise OracleError(rc, "tau")
    return out


def tau_at(delta, vpec, dv, T0, gamma, offsets, skewer, targets, tau_ref=1.0,
           delta_pivot=10.0):
    """Raw optical depth of eq. (6) at the pixels ``targets`` of one skewer
    (the full sum, as ``tau`` with window_k = 0; float64 [len(targets)])."""
    delta, vpec = _d(delta).ravel(), _d(vpec).ravel()
    P = delta.size
    S = len(offsets) - 1
    off = _offsets(S, P, offsets)
    dv_, T0_, g_ = _per_skewer(dv, S), _per_skewer(T0, S), _per_skewer(gamma, S)
    tg = np.ascontiguousarray(targets, np.int64)
    out = np.empty(tg.size, np.float64)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    rc = _load().oracle_tau_at(S, off.ctypes.data_as(pi64), _p(delta), _p(vpec), _p(dv_),
                               _p(T0_), _p(g_), float(tau_ref), float(delta_pivot),
                               int(skewer), tg.ctypes.data_as(pi64), tg.size, _p(out))
    if rc:
        raise OracleError(rc, "tau_at")
    return out


def mean_flux_A(tau_raw, target_F):
    """A such that (1/P) sum exp(-A tau) = target_F; returns (A, iterations)."""
    t = _d(tau_raw).ravel()
    A = ctypes.c_double()
    it = ctypes.c_int()
    rc = _load().oracle_mean_flux_A(t.size, _p(t), float(target_F),
                                    ctypes.byref(A), ctypes.byref(it))
    if rc:
        raise OracleError(rc, "mean_flux_A")
    return A.value, it.value


def finalise(tau_raw, A):
    """(tau' = A tau, F = exp(-tau'))."""
    t = _d(tau_raw).ravel()
    ts = np.empty_like(t)
    F = np.empty_like(t)
    _load().oracle_finalise(t.size, _p(t), float(A), _p(ts), _p(F))
    return ts, F


def normalise(tau_raw, target_F):
    """Mean-flux rescale: returns (tau', F, A)."""
    A, _ = mean_flux_A(tau_raw, target_F)
    ts, F = finalise(tau_raw, A)
    return ts, F, A


def tau_grad(delta, vpec, dv, T0, gamma, g, offsets=None, n_skewers=None,
             tau_ref=1.0, delta_pivot=10.0):
    """Given g = dL/dtau_raw [P], return (dL/dDelta [P], dL/dv [P],
    dL/dT0 [S], dL/dgamma [S])."""
    delta, vpec, g = _d(delta).ravel(), _d(vpec).ravel(), _d(g).ravel()
    P = delta.size
    if offsets is None and n_skewers is None:
        n_skewers = 1
    S = (len(offsets) - 1) if offsets is not None else int(n_skewers)
    off = _offsets(S, P, offsets)
    dv_, T0_, g_ = _per_skewer(dv, S), _per_skewer(T0, S), _per_skewer(gamma, S)
    gd, gv = np.empty(P), np.empty(P)
    gT, gg = np.empty(S), np.empty(S)
    rc = _load().oracle_tau_grad(S, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 _p(delta), _p(vpec), _p(dv_), _p(T0_), _p(g_),
                                 float(tau_ref), float(delta_pivot), _p(g),
                                 _p(gd), _p(gv), _p(gT), _p(gg))
    if rc:
        raise OracleError(rc, "tau_grad")
    return gd, gv, gT, gg


def normalise_backward(tau_raw, A, grad_F=None, grad_tau_scaled=None,
                       implicit_A=True):
    """dL/dtau_raw from dL/dF and dL/dtau' through the mean-flux rescale."""
    t = _d(tau_raw).ravel()
    gF = None if grad_F is None else _d(grad_F).ravel()
    gT = None if grad_tau_scaled is None else _d(grad_tau_scaled).ravel()
    out = np.empty_like(t)
    null = ctypes.POINTER(ctypes.c_double)()
    rc = _load().oracle_normalise_backward(
        t.size, _p(t), float(A), _p(gF) if gF is not None else null,
        _p(gT) if gT is not None else null, int(bool(implicit_A)), _p(out))
    if rc:
        raise OracleError(rc, "normalise_backward")
    return out


def angstrom_to_kms(dlambda, z):
    """Velocity width of ``dlambda`` Angstrom at Lyman alpha observed at ``z``."""
    return float(_load().oracle_angstrom_to_kms(float(dlambda), float(z)))


def lya_lyb_path_kms(proximity_kms=3000.0):
    """Lya-Lyb path length in km/s minus the proximity zone."""
    return float(_load().oracle_lya_lyb_path_kms(float(proximity_kms)))


def lsf_b(fwhm):
    """Width b of exp(-(d/b)^2) with the given FWHM."""
    return float(_load().oracle_lsf_b(float(fwhm)))


def _i64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def instrument(F, offsets, dv, out_offsets, fwhm, bin_kms, v_start=0.0, noise=None,
               sigma=0.0):
    """Mock observation of each skewer's flux: Gaussian line-spread convolution,
    resampling onto ``bin_kms`` bins from ``v_start``, plus ``sigma * noise``.
    Skewer s yields ``out_offsets[s+1] - out_offsets[s]`` bins (float64)."""
    F = _d(F).ravel()
    off = _offsets(None, F.size, offsets)
    S = len(off) - 1
    oo = _offsets(None, 0, out_offsets)
    dv_ = _per_skewer(dv, S)
    out = np.empty(int(oo[-1]), np.float64)
    nz = _d(noise).ravel() if noise is not None else None
    rc = _load().oracle_instrument(S, _i64p(off), _p(F), _p(dv_), float(fwhm), float(bin_kms),
                                   float(v_start), _i64p(oo),
                                   _p(nz) if nz is not None else ctypes.POINTER(ctypes.c_double)(),
                                   float(sigma), _p(out))
    if rc:
        raise OracleError(rc, "instrument")
    return out


def instrument_backward(grad_out, offsets, dv, out_offsets, fwhm, bin_kms, v_start=0.0):
    """dL/dF [P] from dL/d(binned flux) [P_out] (float64)."""
    off = _offsets(None, 0, offsets)
    S = len(off) - 1
    oo = _offsets(None, 0, out_offsets)
    g = _d(grad_out).ravel()
    dv_ = _per_skewer(dv, S)
    out = np.empty(int(off[-1]), np.float64)
    rc = _load().oracle_instrument_backward(S, _i64p(off), _p(dv_), float(fwhm), float(bin_kms),
                                            float(v_start), _i64p(oo), _p(g), _p(out))
    if rc:
        raise OracleError(rc, "instrument_backward")
    return out
