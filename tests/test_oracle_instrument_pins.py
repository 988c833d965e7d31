"""Pins of the instrument-model oracle (Gaussian line-spread convolution,
resampling onto coarser bins, noise) to facts fixed by the paper and by
mathematics.

Each check compares the oracle with something other than its own formula: the
paper's printed Angstrom/km-s pair, the half-maximum width of the measured
impulse response, the closed form for a Gaussian through a Gaussian (widths add
in quadrature), numpy's FFT, numpy's interpolation of the cumulative integral,
block means, conservation and invariance laws, and the dot-product identity of
a linear map with its adjoint.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def paper():
    with open(os.path.join(GOLDEN, "paper_instrument.json")) as f:
        return json.load(f)


def one(F, dv, fwhm, bin_kms, v_start, n_out, noise=None, sigma=0.0):
    F = np.asarray(F, float)
    return O.instrument(F, [0, F.size], dv, [0, n_out], fwhm, bin_kms, v_start, noise, sigma)


def identity_bins(F, dv, fwhm):
    """Bins that coincide with the pixels: the convolved spectrum itself."""
    return one(F, dv, fwhm, dv, -0.5 * dv, len(F))


def test_printed_boss_resolution_pair():
    p = paper()
    b = p["boss"]
    kms = O.angstrom_to_kms(b["fwhm_angstrom"], p["redshift"])
    assert abs(kms - b["fwhm_kms_printed"]) <= 0.5 * 10.0 ** (-b["printed_decimals_kms"])


def test_lya_lyb_path_is_the_integral_of_c_dlambda_over_lambda():
    # velocity along a spectrum: dv = c dlambda / lambda, from Lyb to Lya
    c, la, lb = 299792.458, 1215.67, 1025.72
    path, _ = integrate.quad(lambda lam: c / lam, lb, la, epsabs=1e-10)
    prox = paper()["boss"]["proximity_kms"]
    assert O.lya_lyb_path_kms(prox) == pytest.approx(path - prox, rel=1e-12)


def test_impulse_response_has_the_stated_fwhm():
    dv, fwhm, N = 0.02, 7.0, 4096
    e = np.zeros(N)
    e[0] = 1.0
    h = identity_bins(e, dv, fwhm)
    h = np.roll(h, N // 2)  # peak at the centre
    u = (np.arange(N) - N // 2) * dv
    half = 0.5 * h.max()
    right = np.nonzero((h[:-1] >= half) & (h[1:] < half))[0][-1]
    left = np.nonzero((h[:-1] < half) & (h[1:] >= half))[0][0]
    # log-quadratic (exact for a Gaussian) interpolation between samples
    def cross(i):
        return u[i] + (math.log(half) - math.log(h[i])) / (math.log(h[i + 1]) - math.log(h[i])) * dv
    assert cross(right) - cross(left) == pytest.approx(fwhm, rel=1e-9)
    assert h.sum() == pytest.approx(1.0, rel=1e-14)


@pytest.mark.parametrize("b1,fwhm,dv", [(5.0, 20.0, 1.0), (8.0, 7.0, 2.0), (30.0, 224.0, 4.0)])
def test_gaussian_line_through_gaussian_lsf(b1, fwhm, dv):
    # a continuous Gaussian of width b1 through a Gaussian of width bL has width
    # sqrt(b1^2 + bL^2) and depth scaled by b1 / sqrt(b1^2 + bL^2); bL comes from
    # the FWHM measured in test_impulse_response_has_the_stated_fwhm.
    N = 4096
    u = np.arange(N) * dv
    u0, a = 0.5 * N * dv + 0.3 * dv, 0.6
    F = 1.0 - a * np.exp(-((u - u0) / b1) ** 2)
    bL = fwhm / (2.0 * math.sqrt(math.log(2.0)))
    bc = math.hypot(b1, bL)
    want = 1.0 - a * (b1 / bc) * np.exp(-((u - u0) / bc) ** 2)
    got = identity_bins(F, dv, fwhm)
    assert np.max(np.abs(got - want)) < 1e-11


@pytest.mark.parametrize("N,dv,fwhm", [(96, 2.0, 13.0), (97, 1.5, 400.0), (64, 3.0, 1e4), (50, 2.0, 0.0)])
def test_convolution_is_circular(N, dv, fwhm):
    rng = np.random.default_rng(N)
    F = rng.random(N)
    e = np.zeros(N)
    e[0] = 1.0
    h = identity_bins(e, dv, fwhm)
    want = np.fft.irfft(np.fft.rfft(F) * np.fft.rfft(h), n=N)
    got = identity_bins(F, dv, fwhm)
    assert np.max(np.abs(got - want)) < 1e-13
    # the response is even (minimal images, d^2 only) and sums to one
    assert np.max(np.abs(h - np.roll(h[::-1], 1))) < 1e-16
    assert h.sum() == pytest.approx(1.0, rel=1e-14)


def test_flat_spectrum_is_unchanged():
    for v_start, bin_kms in [(0.0, 3.08), (-137.2, 63.96), (9000.0, 17.0)]:
        out = one(np.full(1000, 0.7), 2.0, 224.0, bin_kms, v_start, int(2000.0 // bin_kms))
        assert np.max(np.abs(out - 0.7)) < 1e-14


@pytest.mark.parametrize("r,shift", [(1, 0), (3, 0), (4, 5), (8, -3)])
def test_aligned_integer_bins_are_block_means(r, shift):
    rng = np.random.default_rng(r)
    N, dv = 96, 2.0
    F = rng.random(N)
    out = one(F, dv, 0.0, r * dv, (shift - 0.5) * dv, N // r)
    want = np.roll(F, -shift).reshape(-1, r).mean(axis=1)
    assert np.max(np.abs(out - want)) < 1e-14


@pytest.mark.parametrize("bin_px,v_start_px", [(2.7, 0.31), (0.77, -5.4), (13.3, 101.9), (1.0, 0.25)])
def test_fractional_bins_integrate_the_piecewise_constant_spectrum(bin_px, v_start_px):
    rng = np.random.default_rng(7)
    N, dv = 120, 2.0
    F = rng.random(N)
    n_out = int(N / bin_px)
    out = one(F, dv, 0.0, bin_px * dv, v_start_px * dv, n_out)
    # cumulative integral at pixel edges over several periods; pixel i covers
    # velocities [(i - 1/2) dv, (i + 1/2) dv)
    laps = 4
    Fl = np.tile(F, laps)
    edges_v = (np.arange(laps * N + 1) - 0.5 - N) * dv
    cum = np.concatenate([[0.0], np.cumsum(Fl * dv)])
    lo = v_start_px * dv + np.arange(n_out) * bin_px * dv
    hi = lo + bin_px * dv
    want = (np.interp(hi, edges_v, cum) - np.interp(lo, edges_v, cum)) / (bin_px * dv)
    assert np.max(np.abs(out - want)) < 1e-12


def test_flux_conservation_when_bins_tile_the_box():
    rng = np.random.default_rng(3)
    N, dv = 500, 2.0
    F = rng.random(N)
    n_out = 37
    bin_kms = N * dv / n_out
    for v_start in (0.0, 123.456, -777.7):
        out = one(F, dv, 170.0, bin_kms, v_start, n_out)
        assert out.sum() * bin_kms == pytest.approx(F.sum() * dv, rel=1e-13)


def test_shift_equivariance():
    rng = np.random.default_rng(4)
    N, dv = 200, 1.7
    F = rng.random(N)
    base = one(F, dv, 30.0, 5.3, 11.0, 50)
    for m in (1, 17, -40):
        got = one(np.roll(F, m), dv, 30.0, 5.3, 11.0 + m * dv, 50)
        assert np.max(np.abs(got - base)) < 1e-13


def test_noise_is_added_with_its_sigma():
    rng = np.random.default_rng(5)
    F = rng.random(300)
    eps = rng.standard_normal(100)
    a = one(F, 2.0, 7.0, 3.08, 0.0, 100)
    b = one(F, 2.0, 7.0, 3.08, 0.0, 100, noise=eps, sigma=1.0 / 50.0)
    assert np.max(np.abs((b - a) - eps / 50.0)) < 1e-15


def test_ragged_skewers_are_independent():
    rng = np.random.default_rng(6)
    lens, nouts = [40, 300, 1000], [10, 0, 120]
    off = np.concatenate([[0], np.cumsum(lens)])
    oo = np.concatenate([[0], np.cumsum(nouts)])
    dvs = np.array([2.0, 1.0, 3.5])
    F = rng.random(off[-1])
    out = O.instrument(F, off, dvs, oo, 70.0, 7.9, -3.0)
    for s in range(3):
        if nouts[s]:
            alone = one(F[off[s]:off[s + 1]], dvs[s], 70.0, 7.9, -3.0, nouts[s])
            assert np.array_equal(out[oo[s]:oo[s + 1]], alone)


def test_backward_is_the_adjoint():
    rng = np.random.default_rng(8)
    lens, nouts = [64, 333, 120], [20, 60, 0]
    off = np.concatenate([[0], np.cumsum(lens)])
    oo = np.concatenate([[0], np.cumsum(nouts)])
    dvs = np.array([2.0, 1.3, 4.0])
    for fwhm, bin_kms, v0 in [(7.0, 3.08, 0.0), (224.0, 6.1, -50.0), (0.0, 1.0, 0.4)]:
        x = rng.standard_normal(off[-1])
        y = rng.standard_normal(oo[-1])
        Jx = O.instrument(x, off, dvs, oo, fwhm, bin_kms, v0)
        JTy = O.instrument_backward(y, off, dvs, oo, fwhm, bin_kms, v0)
        assert float(y @ Jx) == pytest.approx(float(JTy @ x), rel=1e-12, abs=1e-12)
    # a skewer with no bins receives no gradient
    assert np.all(JTy[off[2]:off[3]] == 0.0)


def test_invalid_arguments():
    F = np.ones(100)
    with pytest.raises(O.OracleError):  # bins longer than the box
        one(F, 2.0, 7.0, 3.0, 0.0, 67)
    with pytest.raises(O.OracleError):
        one(F, 2.0, -1.0, 3.0, 0.0, 10)
    with pytest.raises(O.OracleError):
        one(F, 2.0, 7.0, 0.0, 0.0, 10)
    with pytest.raises(O.OracleError):  # noise scale without draws
        one(F, 2.0, 7.0, 3.0, 0.0, 10, sigma=0.1)
