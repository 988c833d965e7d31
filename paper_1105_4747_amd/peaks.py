"""ctypes binding of libpeaks.so: measured FP32 FMA, exp2 and copy rates of the
current device (see include/lyaf_peaks.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpeaks.so")
MIX_N = 6  # LYAF_PEAKS_MIX_N


class PeakRates(ctypes.Structure):
    _fields_ = [("fma_lane_ops_per_s", ctypes.c_double),
                ("pair_per_s_exp", ctypes.c_double),
                ("pair_per_s_noexp", ctypes.c_double),
                ("c_valu_s", ctypes.c_double),
                ("c_exp_s", ctypes.c_double),
                ("pair_peak_per_s", ctypes.c_double),
                ("trans_lane_ops_per_s", ctypes.c_double),
                ("mix_fma_per_exp", ctypes.c_double * MIX_N),
                ("mix_exp_per_s", ctypes.c_double * MIX_N),
                ("copy_bytes_per_s", ctypes.c_double),
                ("compute_units", ctypes.c_int32),
                ("clock_khz", ctypes.c_int32)]


EXPORTED = ["lyaf_peaks_measure"]
_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        from . import build as _build
        if _build.built_hash(LIB_PATH) != _build.source_hash(
                _build.PEAKS_SOURCES + [os.path.join(_build.ROOT, "include", "lyaf_peaks.h")]):
            raise RuntimeError(f"{LIB_PATH} was not built from the current sources: rebuild it")
        lib = ctypes.CDLL(LIB_PATH)
        lib.lyaf_peaks_measure.argtypes = [ctypes.POINTER(PeakRates), ctypes.c_void_p]
        lib.lyaf_peaks_measure.restype = ctypes.c_int
        _lib = lib
    return _lib


def measure(stream=None) -> dict:
    r = PeakRates()
    h = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    rc = load().lyaf_peaks_measure(ctypes.byref(r), h)
    if rc != 0:
        raise RuntimeError(f"lyaf_peaks_measure failed ({rc})")
    out = {}
    for f, _ in PeakRates._fields_:
        v = getattr(r, f)
        out[f] = list(v) if isinstance(v, ctypes.Array) else v
    return out
