"""Pins of the flux-statistics oracle (flux PDF, 1D flux power spectrum) to the
paper's bin layout, numpy's histogram, the plain DFT, Parseval's identity and
single modes."""
import json
import os

import numpy as np
import pytest

from oracle import flux_stats as FS

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_pdf_layout_is_the_papers():
    with open(os.path.join(GOLDEN, "paper_flux_pdf.json")) as f:
        g = json.load(f)
    assert FS.N_PDF_BINS == g["n_bins"] and FS.PDF_BIN_WIDTH == g["bin_width"]
    # centres 0 .. 1, first bin [-0.025, 0.025)
    probes = {0.0: 0, 1.0: 20, 0.024: 0, 0.026: 1, -0.024: 0, 0.5: 10, 0.524: 10,
              0.526: 11, 1.024: 20}
    for F, j in probes.items():
        assert FS.pdf_bin_index([F])[0] == j, F
    assert FS.pdf_bin_index([-0.026])[0] == -1
    assert FS.pdf_bin_index([1.026])[0] == FS.N_PDF_BINS
    assert FS.pdf_bin_index([float("nan")])[0] == -2
    assert FS.pdf_bin_index([float("inf")])[0] == FS.N_PDF_BINS
    assert FS.pdf_bin_index([-float("inf")])[0] == -1


def test_pdf_matches_numpy_histogram_away_from_edges():
    rng = np.random.default_rng(1)
    F = rng.uniform(-0.2, 1.2, 200000).astype(np.float32)
    edges = -0.025 + 0.05 * np.arange(22)
    # keep values clear of every edge so the two edge conventions cannot differ
    d = np.min(np.abs(F.astype(np.float64)[:, None] - edges[None, :]), axis=1)
    F = F[d > 1e-6]
    counts = FS.flux_pdf(F)
    h, _ = np.histogram(F.astype(np.float64), bins=edges)
    assert np.array_equal(counts[:21], h)
    assert counts[FS.PDF_BELOW] == np.count_nonzero(F < edges[0])
    assert counts[FS.PDF_ABOVE] == np.count_nonzero(F >= edges[-1])
    assert counts.sum() == F.size
    dens = FS.pdf_density(counts)
    assert dens.sum() * 0.05 == pytest.approx(1.0, rel=1e-12)


def test_pdf_counts_every_value_once():
    F = np.array([0.1, float("nan"), -5.0, 7.0, 0.95, 1.0, 0.0], np.float32)
    c = FS.flux_pdf(F)
    assert c.sum() == F.size
    assert c[FS.PDF_NAN] == 1 and c[FS.PDF_BELOW] == 1 and c[FS.PDF_ABOVE] == 1
    assert c[2] == 1 and c[19] == 1 and c[20] == 1 and c[0] == 1


@pytest.mark.parametrize("n", [2, 8, 64, 100])
def test_power_is_the_plain_dft(n):
    rng = np.random.default_rng(n)
    F = rng.random(n)
    dv, Fbar = 1.7, 0.7
    P, k = FS.flux_power(F, [0, n], dv, Fbar)
    delta = F / Fbar - 1.0
    j = np.arange(n)
    for m in range(n // 2 + 1):
        X = np.sum(delta * np.exp(-2j * np.pi * m * j / n))
        assert P[m] == pytest.approx(dv / n * abs(X) ** 2, rel=1e-12, abs=1e-15)
        assert k[m] == pytest.approx(2 * np.pi * m / (n * dv), rel=1e-15)


def test_power_parseval():
    rng = np.random.default_rng(2)
    n, dv, Fbar = 4096, 2.0, 0.8
    F = rng.random(n)
    P, _ = FS.flux_power(F, [0, n], dv, Fbar)
    w = np.full(n // 2 + 1, 2.0)
    w[0] = w[-1] = 1.0
    delta = F / Fbar - 1.0
    assert np.sum(w * P) == pytest.approx(dv * np.sum(delta ** 2), rel=1e-12)


@pytest.mark.parametrize("m0", [1, 17, 1000])
def test_power_of_a_single_cosine(m0):
    n, dv, Fbar, A = 4096, 2.0, 0.75, 0.3
    j = np.arange(n)
    F = Fbar * (1.0 + A * np.cos(2 * np.pi * m0 * j / n))
    P, _ = FS.flux_power(F, [0, n], dv, Fbar)
    assert P[m0] == pytest.approx(dv * A * A * n / 4.0, rel=1e-12)
    others = np.delete(P, m0)
    assert np.max(others) < 1e-20 * P[m0] * n


def test_power_of_a_flat_spectrum_is_zero():
    P, _ = FS.flux_power(np.full(512, 0.8), [0, 512], 2.0, 0.8)
    assert np.max(np.abs(P)) == 0.0


def test_power_ragged_skewers_are_independent():
    rng = np.random.default_rng(3)
    lens = [64, 512, 2]
    off = np.concatenate([[0], np.cumsum(lens)])
    F = rng.random(off[-1])
    dvs = np.array([1.0, 2.0, 3.0])
    P, k = FS.flux_power(F, off, dvs, 0.7)
    mo = FS.mode_offsets(off)
    for s in range(3):
        Ps, ks = FS.flux_power(F[off[s]:off[s + 1]], [0, lens[s]], dvs[s], 0.7)
        assert np.array_equal(P[mo[s]:mo[s + 1]], Ps) and np.array_equal(k[mo[s]:mo[s + 1]], ks)
