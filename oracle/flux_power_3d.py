"""FP64 oracle of the 3D flux power spectrum reconstructed from sight-lines --
test infrastructure.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; the product library never does, and this
module imports nothing from the product package.

What it computes (Greig, Bolton & Wyithe 2011, Section 6.2, eq. 7): a mock
survey's S sight-lines of n pixels run along z through columns (x_s, y_s) of
an n^3 periodic grid of side L; the flux contrast delta_s(z) = F_s(z)/F_mean - 1
of each is placed in its column (weight w_s, 1 in the paper), the rest of the
box is empty.  With the unnormalised DFT conventions

  G_s(kz)   = sum_z delta_s(z) e^{-2 pi i kz z / n},
  W(kx, ky) = sum_s w_s e^{-2 pi i (kx x_s + ky y_s) / n},
  D(k)      = sum_s w_s G_s(kz) e^{-2 pi i (kx x_s + ky y_s) / n},

the three power spectra of eq. (7) are

  P_box(k)     = (L^3 / n^6) |D(k)|^2          (the sparse box's 3D power),
  P_1D(kz)     = (L / n^2) mean_s |G_s(kz)|^2   (the mean 1D flux power),
  P_2D,w(kperp) = (L^2 / n^4) |W(kx, ky)|^2    (the weight field's 2D power),

and the reconstruction is P_true(k) = P_box(k) - [P_1D(kz) + P_N] P_2D,w(kperp),
P_N a flat 1D noise power (0 for noiseless spectra).  With these
normalisations the subtracted term equals P_box exactly when every sight-line
carries the same spectrum, which is the aliasing the term removes.  The
spherical average bins the modes of the half-spectrum (kz = 0 .. n/2, each
mode with 0 < kz < n/2 standing also for its conjugate partner, weight 2) by
|m| = sqrt(mx^2 + my^2 + mz^2) (k = 2 pi m / L): bin b holds b <= |m| < b + 1,
shells between consecutive multiples of the fundamental 2 pi / L; each bin
reports its mode count, the mean |k| of its modes and the mean P_true and
P_box.  Reading of the paper's "multiples of the Nyquist frequency": the
shells are spaced by the fundamental mode (multiples of the Nyquist
wavenumber pi n / L would leave two bins).

Parity status: pinned by brute-force DFT sums on small grids, identical
sight-lines (P_true = 0), a single sight-line (P_true = -P_N L^2 / n^4),
Parseval's identity for the box, brute-force shell counts, and linearity in P_N.
"""
from __future__ import annotations

import numpy as np


def contrast(F, mean_F):
    return np.asarray(F, np.float64) / float(mean_F) - 1.0


def line_spectra(delta):
    """G_s(kz), kz = 0 .. n/2, for delta [S, n]."""
    return np.fft.rfft(np.asarray(delta, np.float64), axis=1)


def mode_grid(n):
    """Signed integer wavenumbers (mx [n], my [n], mz [n/2+1])."""
    m = np.fft.fftfreq(n, d=1.0 / n)
    return m, m, np.arange(n // 2 + 1, dtype=np.float64)


def box_spectrum(G, sx, sy, w, n):
    """D(kx, ky, kz) [n, n, n/2+1] and W(kx, ky) [n, n]: the sight-lines'
    contributions scattered into their columns, then 2D FFTs per kz plane."""
    S = G.shape[0]
    grid = np.zeros((n, n, n // 2 + 1), np.complex128)
    wg = np.zeros((n, n), np.float64)
    for s in range(S):
        grid[sx[s], sy[s], :] += w[s] * G[s]
        wg[sx[s], sy[s]] += w[s]
    D = np.fft.fft2(grid, axes=(0, 1))
    W = np.fft.fft2(wg)
    return D, W


def reconstruct(F, mean_F, sx, sy, n, L, weights=None, p_noise=0.0):
    """P_true, P_box [n, n, n/2+1], P_1D [n/2+1] and P_2D,w [n, n] (eq. 7)."""
    delta = contrast(F, mean_F).reshape(len(sx), n)
    w = np.ones(len(sx)) if weights is None else np.asarray(weights, np.float64)
    G = line_spectra(delta)
    D, W = box_spectrum(G, sx, sy, w, n)
    P_box = L ** 3 / n ** 6 * np.abs(D) ** 2
    P_1d = L / n ** 2 * np.mean(np.abs(G) ** 2, axis=0)
    P_2d = L ** 2 / n ** 4 * np.abs(W) ** 2
    P_true = P_box - (P_1d[None, None, :] + p_noise) * P_2d[:, :, None]
    return P_true, P_box, P_1d, P_2d


def shell_average(P_true, P_box, n, L, n_bins):
    """Spherical shells of width 2 pi / L over the half-spectrum: counts, mean
    |k|, mean P_true, mean P_box per bin (float64 [n_bins] each)."""
    mx, my, mz = mode_grid(n)
    m = np.sqrt(mx[:, None, None] ** 2 + my[None, :, None] ** 2 + mz[None, None, :] ** 2)
    c = np.where((mz == 0) | (mz == n // 2), 1.0, 2.0)[None, None, :] * np.ones_like(m)
    b = np.floor(m).astype(np.int64)
    keep = b < n_bins
    cnt = np.bincount(b[keep], weights=c[keep], minlength=n_bins)
    ks = np.bincount(b[keep], weights=(c * m)[keep], minlength=n_bins)
    pt = np.bincount(b[keep], weights=(c * P_true)[keep], minlength=n_bins)
    pb = np.bincount(b[keep], weights=(c * P_box)[keep], minlength=n_bins)
    with np.errstate(invalid="ignore", divide="ignore"):
        return (cnt, np.where(cnt > 0, ks / cnt, 0.0) * (2 * np.pi / L),
                np.where(cnt > 0, pt / cnt, 0.0), np.where(cnt > 0, pb / cnt, 0.0))


def flux_power_3d(F, mean_F, sx, sy, n, L, n_bins, weights=None, p_noise=0.0):
    """The binned reconstruction: (counts, k_mean, P_true_mean, P_box_mean)."""
    P_true, P_box, _, _ = reconstruct(F, mean_F, sx, sy, n, L, weights, p_noise)
    return shell_average(P_true, P_box, n, L, n_bins)
