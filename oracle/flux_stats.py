"""FP64 oracle for the flux statistics of Greig, Bolton & Wyithe (2011), Section 4
-- test infrastructure.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; the product library never does.  It
imports nothing from the product package and shares no code with it.

Flux PDF (Section 4.2).  The transmitted flux is counted in 21 bins of width
0.05 centred on F = 0, 0.05, ..., 1: bin j holds 0.05 j - 0.025 <= F <
0.05 j + 0.025.  Here the bin is j = floor((F + 0.025) * 20) evaluated in IEEE
double precision on the (exact) double value of the input, one rounding after
the addition and one after the product; a value below the first bin, at or
above the end of the last, or not a number is counted apart.  The library takes
the same decision in the same precision, so the counts must agree exactly.

1D flux power spectrum (Section 4.3).  The paper compares the line-of-sight
power of the flux with measurements but prints no estimator; the standard one
is used.  Per skewer of N pixels of width dv, with delta_j = F_j / Fbar - 1
(Fbar the mean flux the caller names, e.g. the target of the rescale),

    P(k_m) = (dv / N) |sum_j delta_j exp(-2 pi i m j / N)|^2,
    k_m = 2 pi m / (N dv),   m = 0 .. N/2,

in km/s (k in s/km).  numpy's real FFT supplies the sum; the pins check it
against the plain DFT, Parseval's identity and single modes.

Parity status: flux_pdf pinned (numpy.histogram away from bin edges, counts
sum to the input size, the paper's bin layout); flux_power pinned (brute-force
DFT, Parseval, a cosine's single mode, a flat spectrum).
"""
from __future__ import annotations

import numpy as np

N_PDF_BINS = 21          # Section 4.2
PDF_BIN_WIDTH = 0.05
PDF_HALF_WIDTH = 0.025
# counts layout: bins 0..20, then below, above, not-a-number
PDF_BELOW, PDF_ABOVE, PDF_NAN = N_PDF_BINS, N_PDF_BINS + 1, N_PDF_BINS + 2
PDF_SLOTS = N_PDF_BINS + 3


def pdf_bin_index(F):
    """Bin index per value (float64 math on the exact input), -1 below,
    21 at or above the end, -2 for NaN."""
    x = np.asarray(F, dtype=np.float64)
    t = (x + PDF_HALF_WIDTH) * (1.0 / PDF_BIN_WIDTH)
    j = np.full(x.shape, -2, dtype=np.int64)
    ok = ~np.isnan(t)
    j[ok & (t < 0.0)] = -1
    j[ok & (t >= N_PDF_BINS)] = N_PDF_BINS
    inside = ok & (t >= 0.0) & (t < N_PDF_BINS)
    j[inside] = np.floor(t[inside]).astype(np.int64)
    return j


def flux_pdf(F):
    """Counts [24]: bins 0..20, below, above, NaN (int64)."""
    j = pdf_bin_index(np.ravel(F))
    out = np.zeros(PDF_SLOTS, np.int64)
    for b in range(N_PDF_BINS):
        out[b] = int(np.count_nonzero(j == b))
    out[PDF_BELOW] = int(np.count_nonzero(j == -1))
    out[PDF_ABOVE] = int(np.count_nonzero(j == N_PDF_BINS))
    out[PDF_NAN] = int(np.count_nonzero(j == -2))
    return out


def pdf_density(counts):
    """Normalised PDF over the 21 bins: counts / (in-range count * 0.05)."""
    c = np.asarray(counts[:N_PDF_BINS], np.float64)
    return c / (c.sum() * PDF_BIN_WIDTH)


def mode_offsets(offsets):
    """Offsets of the per-skewer mode arrays: skewer s holds N_s/2 + 1 modes."""
    n = np.diff(np.asarray(offsets, np.int64))
    return np.concatenate([[0], np.cumsum(n // 2 + 1)]).astype(np.int64)


def flux_power(F, offsets, dv, mean_F):
    """Per-skewer power P(k_m), m = 0 .. N_s/2, concatenated (float64), and
    the matching k_m (s/km)."""
    F = np.asarray(F, np.float64).ravel()
    off = np.asarray(offsets, np.int64)
    S = len(off) - 1
    dv = np.broadcast_to(np.asarray(dv, np.float64), (S,))
    mo = mode_offsets(off)
    P = np.empty(int(mo[-1]), np.float64)
    k = np.empty_like(P)
    for s in range(S):
        n = int(off[s + 1] - off[s])
        delta = F[off[s]:off[s + 1]] / float(mean_F) - 1.0
        X = np.fft.rfft(delta)
        P[mo[s]:mo[s + 1]] = (dv[s] / n) * (X.real ** 2 + X.imag ** 2)
        k[mo[s]:mo[s + 1]] = 2.0 * np.pi * np.arange(n // 2 + 1) / (n * dv[s])
    return P, k
