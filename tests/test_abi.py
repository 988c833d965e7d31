"""CPU checks of the C ABI: the library loads, exports every function that
include/lyaf.h declares, and rejects bad arguments on the host before touching
the GPU (no compute call is made here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1105_4747_amd import lyaf as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lyaf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|double|const char \*)\s*(lyaf_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert {"lyaf_tau", "lyaf_normalise_mean_flux", "lyaf_tau_backward"} <= set(names)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in lyaf.h but not exported"
    assert set(L.EXPORTED) == set(names)


def test_version_and_strerror(lib):
    assert L.version() >= 100
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.strerror(code)
    assert L.strerror(-99) == "unknown error"


def _call_tau(off, tau_ref=1.0, pivot=10.0, k=6.0, S=None, ptrs=True, out=True):
    off = np.asarray(off, np.int64)
    dummy = ctypes.c_void_p(0x1000) if ptrs else None  # never dereferenced: validation fails first
    sk = L.Skewers(len(off) - 1 if S is None else S,
                   off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                   dummy, dummy, dummy, dummy, dummy)
    prm = L.Params(tau_ref, pivot, k, 0)
    return L.load().lyaf_tau(ctypes.byref(sk), ctypes.byref(prm),
                             ctypes.c_void_p(0x2000) if out else None, None)


@pytest.mark.parametrize("kw", [
    dict(off=[0, 10], tau_ref=0.0),
    dict(off=[0, 10], tau_ref=-1.0),
    dict(off=[0, 10], tau_ref=float("nan")),
    dict(off=[0, 10], pivot=0.0),
    dict(off=[0, 10], k=-1.0),
    dict(off=[0, 10], k=float("inf")),
    dict(off=[1, 10]),                 # offsets[0] != 0
    dict(off=[0, 10, 5]),              # decreasing
    dict(off=[0, (1 << 24) + 1]),      # skewer longer than 2^24 pixels
    dict(off=[0, 10], S=-1),
    dict(off=[0, 10], ptrs=False),     # null device arrays
    dict(off=[0, 10], out=False),      # null output
])
def test_tau_rejects_bad_arguments_on_host(kw):
    assert _call_tau(**kw) == L.LYAF_EINVAL


def test_tau_null_structs(lib):
    prm = L.Params(1.0, 10.0, 6.0, 0)
    assert lib.lyaf_tau(None, ctypes.byref(prm), None, None) == L.LYAF_EINVAL
    off = np.array([0, 4], np.int64)
    sk = L.Skewers(1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), *([None] * 5))
    assert lib.lyaf_tau(ctypes.byref(sk), None, None, None) == L.LYAF_EINVAL


def test_empty_batch_is_a_no_op(lib):
    # S = 0 and all-empty skewers: nothing to do, nothing enqueued
    assert _call_tau([0], S=0, ptrs=False, out=False) == L.LYAF_OK
    assert _call_tau([0, 0, 0], out=False) == L.LYAF_OK


def test_normalise_rejects_bad_arguments(lib):
    p = ctypes.c_void_p(0x1000)
    q = ctypes.c_void_p(0x3000)
    A = ctypes.c_void_p(0x2000)
    f = lib.lyaf_normalise_mean_flux
    assert f(0, p, q, 0.5, A, None) == L.LYAF_EINVAL        # empty
    assert f(-3, p, q, 0.5, A, None) == L.LYAF_EINVAL
    assert f(10, None, q, 0.5, A, None) == L.LYAF_EINVAL
    assert f(10, p, q, 0.5, None, None) == L.LYAF_EINVAL
    assert f(10, p, p, 0.5, A, None) == L.LYAF_EINVAL       # F aliases tau
    for F in (0.0, 1.0, -0.1, 1.5, float("nan")):
        assert f(10, p, q, F, A, None) == L.LYAF_EINVAL
    n = lib.lyaf_normalise_mean_flux_noalloc
    assert n(0, p, q, 0.5, A, None, None) == L.LYAF_EINVAL
    assert n(-3, p, q, 0.5, A, None, None) == L.LYAF_EINVAL
    assert n(10, None, q, 0.5, A, None, None) == L.LYAF_EINVAL
    assert n(10, p, q, 0.5, None, None, None) == L.LYAF_EINVAL
    assert n(10, p, p, 0.5, A, None, None) == L.LYAF_EINVAL
    assert n((1 << 48) + 1, p, q, 0.5, A, None, None) == L.LYAF_EINVAL   # beyond the maximum
    assert f((1 << 48) + 1, p, q, 0.5, A, None) == L.LYAF_EINVAL
    for F in (0.0, 1.0, -0.1, 1.5, float("nan")):
        assert n(10, p, q, F, A, None, None) == L.LYAF_EINVAL
    b = lib.lyaf_normalise_mean_flux_backward
    assert b(-1, p, A, None, None, 1, q, None) == L.LYAF_EINVAL
    assert b(10, None, A, None, None, 1, q, None) == L.LYAF_EINVAL
    assert b(0, None, None, None, None, 1, None, None) == L.LYAF_OK


def test_tau_backward_rejects_bad_arguments(lib):
    off = np.array([0, 10], np.int64)
    d = ctypes.c_void_p(0x1000)
    sk = L.Skewers(1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), d, d, d, d, d)
    prm = L.Params(1.0, 10.0, 6.0, 0)
    f = lib.lyaf_tau_backward
    assert f(ctypes.byref(sk), ctypes.byref(prm), None, d, d, None, None, None) == L.LYAF_EINVAL
    assert f(ctypes.byref(sk), ctypes.byref(prm), d, None, d, None, None, None) == L.LYAF_EINVAL
    bad = L.Params(-1.0, 10.0, 6.0, 0)
    assert f(ctypes.byref(sk), ctypes.byref(bad), d, d, d, None, None, None) == L.LYAF_EINVAL
    assert lib.lyaf_status_read(None, None) == L.LYAF_EINVAL


def test_plan_create_rejects_bad_arguments(lib):
    off = np.array([0, 10], np.int64)
    d = ctypes.c_void_p(0x1000)
    sk = L.Skewers(1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), d, d, d, d, d)
    prm = L.Params(1.0, 10.0, 6.0, 0)
    h = ctypes.c_void_p()
    f = lib.lyaf_plan_create
    o, F, A = ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000)
    assert f(ctypes.byref(sk), ctypes.byref(prm), 0.8, o, F, A, 0, None, None) == L.LYAF_EINVAL
    assert f(ctypes.byref(sk), ctypes.byref(prm), 1.2, o, F, A, 0, None,
             ctypes.byref(h)) == L.LYAF_EINVAL
    assert f(ctypes.byref(sk), ctypes.byref(prm), 0.8, o, o, A, 0, None,
             ctypes.byref(h)) == L.LYAF_EINVAL
    assert f(ctypes.byref(sk), ctypes.byref(prm), 0.8, o, F, None, 0, None,
             ctypes.byref(h)) == L.LYAF_EINVAL
    assert f(ctypes.byref(sk), ctypes.byref(prm), 0.8, o, F, A, 64, None,
             ctypes.byref(h)) == L.LYAF_EINVAL
    assert lib.lyaf_plan_execute(None, None) == L.LYAF_EINVAL
    assert lib.lyaf_plan_destroy(None) == L.LYAF_OK
    assert lib.lyaf_plan_describe(None, None, 0) == L.LYAF_EINVAL
    bad = L.Params(1.0, 10.0, 6.0, L.FLAG_SHAPE(L.NUM_SHAPES))
    assert lib.lyaf_tau(ctypes.byref(sk), ctypes.byref(bad), o, None) == L.LYAF_EINVAL


def test_library_does_not_link_the_oracle():
    """The product library and its binding reference nothing under oracle/."""
    pkg = os.path.join(ROOT, "paper_1105_4747_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "oracle" not in txt.lower(), f"{fn} mentions the oracle"
    so = open(L.library_path(), "rb").read()
    assert b"oracle_" not in so


def test_peaks_library_exports_and_rejects_null():
    """libpeaks.so (the benchmark's rate microbenchmarks) exports what
    include/lyaf_peaks.h declares; a null output is rejected before any
    device call."""
    from paper_1105_4747_amd import peaks
    src = open(os.path.join(ROOT, "include", "lyaf_peaks.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = sorted(set(re.findall(r"^\s*int\s+(lyaf_\w+)\s*\(", src, re.M)))
    lib = peaks.load()
    assert names == sorted(peaks.EXPORTED)
    for n in names:
        assert hasattr(lib, n)
    assert lib.lyaf_peaks_measure(None, None) == -1


def _ins(lib, off=(0, 10), oo=(0, 4), fwhm=7.0, bin_kms=3.0, v0=0.0, sigma=0.0, k=6.0,
         ptrs=True, noise=False, S=None, backward=False):
    off = np.asarray(off, np.int64)
    oo = np.asarray(oo, np.int64)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    d = ctypes.c_void_p(0x1000) if ptrs else None  # never dereferenced: validation fails first
    ip = L.InstrumentParams(fwhm, bin_kms, v0, sigma, k)
    n = len(off) - 1 if S is None else S
    if backward:
        return lib.lyaf_instrument_backward(n, off.ctypes.data_as(pi64), d, ctypes.byref(ip),
                                            oo.ctypes.data_as(pi64), d, d, None)
    return lib.lyaf_instrument(n, off.ctypes.data_as(pi64), d, d, ctypes.byref(ip),
                               oo.ctypes.data_as(pi64), ctypes.c_void_p(0x3000) if noise else None,
                               d, None)


@pytest.mark.parametrize("backward", [False, True])
@pytest.mark.parametrize("kw", [
    dict(fwhm=-1.0), dict(fwhm=float("nan")), dict(bin_kms=0.0), dict(bin_kms=float("inf")),
    dict(v0=float("nan")), dict(sigma=-0.1), dict(k=-1.0), dict(S=-1),
    dict(off=(1, 10)), dict(oo=(1, 4)), dict(off=(0, 10, 5), oo=(0, 4, 4)),
    dict(off=(0, 10, 10), oo=(0, 4, 6)),  # bins for an empty skewer
    dict(oo=(0, -1)), dict(ptrs=False),
])
def test_instrument_rejects_bad_arguments_on_host(lib, kw, backward):
    assert _ins(lib, backward=backward, **kw) == L.LYAF_EINVAL


def test_instrument_noise_and_empty_cases(lib):
    # a noise scale needs the draws
    assert _ins(lib, sigma=0.02) == L.LYAF_EINVAL
    # nothing to do: no bins (forward) / no pixels (backward)
    assert _ins(lib, oo=(0, 0)) == L.LYAF_OK
    assert _ins(lib, off=(0,), oo=(0,), S=0, ptrs=False, backward=True) == L.LYAF_OK


def test_instrument_unit_conversions_match_the_paper(lib):
    # Section 3.2 prints the BOSS-like resolution as ~3.63 A and ~224 km/s at z = 3
    assert abs(L.angstrom_to_kms(3.63, 3.0) - 224.0) < 0.5
    assert L.angstrom_to_kms(1.0375, 3.0) == pytest.approx(63.9636, rel=1e-5)
    assert 47000.0 < L.lya_lyb_path_kms(3000.0) < 49000.0


def test_flux_pdf_rejects_bad_arguments(lib):
    p = ctypes.c_void_p(0x1000)
    f = lib.lyaf_flux_pdf
    assert f(-1, p, p, None) == L.LYAF_EINVAL
    assert f(10, None, p, None) == L.LYAF_EINVAL
    assert f(10, p, None, None) == L.LYAF_EINVAL


@pytest.mark.parametrize("lens,mean_F", [
    ([3], 0.8), ([1], 0.8), ([0], 0.8), ([16384], 0.8), ([4096, 100], 0.8),
    ([64], 0.0), ([64], -1.0), ([64], float("nan")), ([64], float("inf")),
])
def test_flux_power_rejects_bad_arguments(lib, lens, mean_F):
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    p = ctypes.c_void_p(0x1000)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    assert lib.lyaf_flux_power(len(lens), off.ctypes.data_as(pi64), p, p, mean_F, p,
                               None) == L.LYAF_EINVAL


def test_flux_power_null_pointers_and_empty(lib):
    off = np.array([0, 64], np.int64)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    p = ctypes.c_void_p(0x1000)
    f = lib.lyaf_flux_power
    assert f(1, off.ctypes.data_as(pi64), None, p, 0.8, p, None) == L.LYAF_EINVAL
    assert f(1, off.ctypes.data_as(pi64), p, None, 0.8, p, None) == L.LYAF_EINVAL
    assert f(1, off.ctypes.data_as(pi64), p, p, 0.8, None, None) == L.LYAF_EINVAL
    assert f(1, None, p, p, 0.8, p, None) == L.LYAF_EINVAL
    assert f(0, None, None, None, 0.8, None, None) == L.LYAF_OK


def test_kernel_timing_records_nothing_when_idle(lib):
    """Kernel timing is host bookkeeping until a launch is recorded: turning it
    on and off and reading a name with no records makes no device call."""
    assert lib.lyaf_kernel_timing_read(None, None, None) == L.LYAF_EINVAL
    L.kernel_timing(True)
    assert L.kernel_timing_read("tau") == (0.0, 0)
    L.kernel_timing(False)
    assert L.kernel_timing_read("tau") == (0.0, 0)


def _field_params(**kw):
    d = dict(n=16, box=10.0, amp=1.0, k_F=2.0, E_plus=50.0, dk=0.1, n_table=8)
    d.update(kw)
    return L.FieldParams(d["n"], d["box"], d["amp"], d["k_F"], d["E_plus"], d["dk"],
                         d["n_table"])


@pytest.mark.parametrize("kw", [dict(n=2), dict(n=12), dict(n=4096), dict(box=0.0),
                                dict(box=float("inf")), dict(amp=float("nan")),
                                dict(k_F=0.0), dict(k_F=-1.0), dict(E_plus=float("inf")),
                                dict(dk=0.0), dict(n_table=0)])
def test_field_skewers_rejects_bad_parameters(lib, kw):
    p = ctypes.c_void_p(0x1000)
    pi32 = ctypes.POINTER(ctypes.c_int32)
    xs = (ctypes.c_int32 * 2)(0, 1)
    fp = _field_params(**kw)
    assert lib.lyaf_field_skewers(ctypes.byref(fp), p, p, 2, ctypes.cast(xs, pi32),
                                  ctypes.cast(xs, pi32), p, p, None) == L.LYAF_EINVAL


def test_field_skewers_rejects_bad_columns_and_pointers(lib):
    p = ctypes.c_void_p(0x1000)
    pi32 = ctypes.POINTER(ctypes.c_int32)
    good = (ctypes.c_int32 * 2)(0, 15)
    f = lib.lyaf_field_skewers
    fp = _field_params()
    for bad in ((0, 16), (-1, 3)):
        b = (ctypes.c_int32 * 2)(*bad)
        assert f(ctypes.byref(fp), p, p, 2, ctypes.cast(b, pi32), ctypes.cast(good, pi32),
                 p, p, None) == L.LYAF_EINVAL
        assert f(ctypes.byref(fp), p, p, 2, ctypes.cast(good, pi32), ctypes.cast(b, pi32),
                 p, p, None) == L.LYAF_EINVAL
    gx = ctypes.cast(good, pi32)
    assert f(None, p, p, 2, gx, gx, p, p, None) == L.LYAF_EINVAL
    assert f(ctypes.byref(fp), None, p, 2, gx, gx, p, p, None) == L.LYAF_EINVAL
    assert f(ctypes.byref(fp), p, None, 2, gx, gx, p, p, None) == L.LYAF_EINVAL
    assert f(ctypes.byref(fp), p, p, 2, None, gx, p, p, None) == L.LYAF_EINVAL
    assert f(ctypes.byref(fp), p, p, 2, gx, gx, None, p, None) == L.LYAF_EINVAL
    assert f(ctypes.byref(fp), p, p, 2, gx, gx, p, None, None) == L.LYAF_EINVAL
    assert f(ctypes.byref(fp), p, p, -1, gx, gx, p, p, None) == L.LYAF_EINVAL
    # no sight-lines: nothing to do, no pointer is read
    assert f(ctypes.byref(fp), None, None, 0, None, None, None, None, None) == L.LYAF_OK
    fp_inf = _field_params(k_F=float("inf"))  # no filter is allowed
    assert f(ctypes.byref(fp_inf), None, None, 0, None, None, None, None, None) == L.LYAF_OK


def _p3d_params(**kw):
    d = dict(n=16, box=10.0, mean_F=0.7, p_noise=0.0, n_bins=20)
    d.update(kw)
    return L.Power3dParams(d["n"], d["box"], d["mean_F"], d["p_noise"], d["n_bins"])


@pytest.mark.parametrize("kw", [dict(n=2), dict(n=24), dict(n=4096), dict(box=0.0),
                                dict(box=float("nan")), dict(mean_F=0.0),
                                dict(mean_F=float("inf")), dict(p_noise=-1.0),
                                dict(p_noise=float("inf")), dict(n_bins=0)])
def test_flux_power_3d_rejects_bad_parameters(lib, kw):
    p = ctypes.c_void_p(0x1000)
    pi32 = ctypes.POINTER(ctypes.c_int32)
    xs = ctypes.cast((ctypes.c_int32 * 2)(0, 1), pi32)
    pp = _p3d_params(**kw)
    assert lib.lyaf_flux_power_3d(ctypes.byref(pp), 2, p, xs, xs, None, p, p, p, p,
                                  None) == L.LYAF_EINVAL


def test_flux_power_3d_rejects_bad_columns_and_pointers(lib):
    p = ctypes.c_void_p(0x1000)
    pi32 = ctypes.POINTER(ctypes.c_int32)
    g = ctypes.cast((ctypes.c_int32 * 2)(0, 15), pi32)
    f = lib.lyaf_flux_power_3d
    pp = _p3d_params()
    for bad in ((0, 16), (-1, 3)):
        b = ctypes.cast((ctypes.c_int32 * 2)(*bad), pi32)
        assert f(ctypes.byref(pp), 2, p, b, g, None, p, p, p, p, None) == L.LYAF_EINVAL
        assert f(ctypes.byref(pp), 2, p, g, b, None, p, p, p, p, None) == L.LYAF_EINVAL
    assert f(None, 2, p, g, g, None, p, p, p, p, None) == L.LYAF_EINVAL
    assert f(ctypes.byref(pp), 0, p, g, g, None, p, p, p, p, None) == L.LYAF_EINVAL
    assert f(ctypes.byref(pp), 2, None, g, g, None, p, p, p, p, None) == L.LYAF_EINVAL
    assert f(ctypes.byref(pp), 2, p, None, g, None, p, p, p, p, None) == L.LYAF_EINVAL
    for k in range(4):
        outs = [p, p, p, p]
        outs[k] = None
        assert f(ctypes.byref(pp), 2, p, g, g, None, *outs, None) == L.LYAF_EINVAL
