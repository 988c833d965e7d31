"""FP64 oracle of the skewer-only field synthesis -- test infrastructure.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; the product library never does, and this
module imports nothing from the product package.

What it computes (Greig, Bolton & Wyithe 2011, Section 2.1 and Appendix B):
a linear dark-matter density field is drawn in Fourier space on an N^3 grid
of a periodic box of side L; the baryon field is the dark-matter field
smoothed by the filter of eq. (1), delta_b(k) = delta_DM(k) / (1 + k^2/k_F^2);
the peculiar velocity follows eq. (3), v(k) = E_+ i k / k^2 delta_DM(k), of
which the component along the sight-lines (z) is kept; and only the
sight-lines that are needed are transformed back to real space.

Inputs, all explicit so that both sides compute the same numbers:
  modes    complex [N, N, N/2+1]: the Gaussian white-noise modes g(k) on the
           half-spectrum of a real field (index order kx, ky, kz; kx and ky
           run 0..N-1 with n > N/2 standing for n - N, kz runs 0..N/2),
  pk       [n_k]: the linear power spectrum tabulated at |k| = j dk,
           j = 0..n_k-1, linearly interpolated, 0 beyond the table,
  amp      scalar: delta_DM(k) = amp sqrt(P(|k|)) g(k) (normalisation),
  L, k_F, E_plus: box side, filtering scale of eq. (1), and the velocity
           factor E_+ of eq. (3),
  sx, sy   [S] integer grid columns of the sight-lines.
with k = (2 pi / L) (nx, ny, nz).  The real field of a half-spectrum F is

  f(x, y, z) = N^-3 sum_{kx, ky} sum_{kz=0}^{N/2} c_kz Re[F(k) e^{2 pi i (kx x + ky y + kz z)/N}]

with c_kz = 1 for kz = 0 and N/2 and 2 otherwise (the Hermitian partners of
the modes with 0 < kz < N/2 are implied); numpy's irfftn computes exactly this.
Outputs: delta_b and v_z on the S sight-lines, float64 [S, N] each.

The plane-by-plane path (``skewer_fields_planes``) serves grids too large for
the full inverse transform and is pinned against ``skewer_fields``.

Parity status: pinned by the explicit sum above (brute force on small grids),
single-mode closed forms for delta_b and v_z, Parseval's identity, the
filter's limit k_F -> infinity, linear interpolation of a table that is linear
in k, and the ratio v_z / delta_DM of a single mode (eq. 3).
"""
from __future__ import annotations

import numpy as np


def wavenumbers(N: int, L: float):
    """kx, ky [N] and kz [N/2+1] in the box's units (2 pi n / L)."""
    n = np.fft.fftfreq(N, d=1.0 / N)  # 0, 1, .., N/2-1, -N/2, .., -1
    nz = np.arange(N // 2 + 1, dtype=np.float64)
    f = 2.0 * np.pi / L
    return f * n, f * n, f * nz


def power_at(kmag, pk, dk):
    """Linear interpolation of the table pk (pk[j] at |k| = j dk), 0 beyond it."""
    pk = np.asarray(pk, np.float64)
    j = np.arange(pk.size) * dk
    return np.interp(kmag, j, pk, right=0.0)


def spectra(modes, pk, dk, amp, L, k_F, E_plus):
    """delta_b(k) (eq. 1) and v_z(k) (z component of eq. 3) on the half-spectrum."""
    N = modes.shape[0]
    kx, ky, kz = wavenumbers(N, L)
    k2 = kx[:, None, None] ** 2 + ky[None, :, None] ** 2 + kz[None, None, :] ** 2
    kmag = np.sqrt(k2)
    dm = amp * np.sqrt(power_at(kmag, pk, dk)) * np.asarray(modes, np.complex128)
    filt = 1.0 / (1.0 + k2 / (k_F * k_F)) if np.isfinite(k_F) else np.ones_like(k2)
    db = dm * filt
    with np.errstate(divide="ignore", invalid="ignore"):
        vk = np.where(k2 > 0, E_plus * 1j * kz[None, None, :] / k2, 0.0) * dm
    return db, vk


def real_field(F):
    """The real N^3 field of a half-spectrum F (the sum in the header)."""
    N = F.shape[0]
    return np.fft.irfftn(F, s=(N, N, N), axes=(0, 1, 2))


def skewer_fields(modes, pk, dk, amp, L, k_F, E_plus, sx, sy):
    """delta_b and v_z along the sight-lines (sx[s], sy[s], z), float64 [S, N]."""
    db, vk = spectra(modes, pk, dk, amp, L, k_F, E_plus)
    sx = np.asarray(sx, np.int64)
    sy = np.asarray(sy, np.int64)
    fb = real_field(db)
    fv = real_field(vk)
    return fb[sx, sy, :], fv[sx, sy, :]


def explicit_sum(F, x, y, z):
    """The header's sum at one point, term by term (for small grids)."""
    N = F.shape[0]
    tot = 0.0
    for a in range(N):
        for b in range(N):
            for c in range(N // 2 + 1):
                w = 1.0 if c in (0, N // 2) else 2.0
                ph = 2.0 * np.pi * (a * x + b * y + c * z) / N
                tot += w * (F[a, b, c] * np.exp(1j * ph)).real
    return tot / N ** 3


def skewer_fields_direct(modes, pk, dk, amp, L, k_F, E_plus, sx, sy, chunk=16):
    """The same outputs as ``skewer_fields`` without forming the real grid:
    for each sight-line, C(kz) = sum_{kx, ky} F(k) e^{2 pi i (kx x + ky y)/n}
    directly, then the sum over kz by numpy's inverse real FFT along z (which
    takes the real part of the kz = 0 and n/2 terms, as the header's sum does).
    For grids too large for a full inverse transform."""
    N = modes.shape[0]
    kx, ky, kz = wavenumbers(N, L)
    k2 = kx[:, None, None] ** 2 + ky[None, :, None] ** 2 + kz[None, None, :] ** 2
    kmag = np.sqrt(k2)
    A = amp * np.sqrt(power_at(kmag, pk, dk))
    filt = 1.0 / (1.0 + k2 / (k_F * k_F)) if np.isfinite(k_F) else 1.0
    with np.errstate(divide="ignore", invalid="ignore"):
        vf = np.where(k2 > 0, E_plus * kz[None, None, :] / k2, 0.0)
    del k2, kmag
    g = np.asarray(modes, np.complex128)
    Fb = A * filt * g
    Fv = 1j * A * vf * g
    del g, A, vf
    n_idx = np.arange(N)
    out_b = np.empty((len(sx), N))
    out_v = np.empty((len(sx), N))
    for s0 in range(0, len(sx), chunk):
        xs = np.asarray(sx[s0:s0 + chunk])
        ys = np.asarray(sy[s0:s0 + chunk])
        ex = np.exp(2j * np.pi * np.outer(xs, n_idx) / N)  # [s, kx]
        ey = np.exp(2j * np.pi * np.outer(ys, n_idx) / N)  # [s, ky]
        Cb = np.einsum("sa,abc,sb->sc", ex, Fb, ey, optimize=True)
        Cv = np.einsum("sa,abc,sb->sc", ex, Fv, ey, optimize=True)
        out_b[s0:s0 + chunk] = np.fft.irfft(Cb, n=N, axis=1) / N ** 2
        out_v[s0:s0 + chunk] = np.fft.irfft(Cv, n=N, axis=1) / N ** 2
    return out_b, out_v


def skewer_fields_planes(modes, pk, dk, amp, L, k_F, E_plus, sx, sy):
    """The same outputs as ``skewer_fields`` for a few sight-lines of a grid
    too large to hold in FP64: one mx plane of the half-spectrum at a time,
    its multipliers (eqs. 1 and 3) formed for that plane only, then
    C_s(mz) += e^{2 pi i mx x_s / N} sum_my e^{2 pi i my y_s / N} F(mx, my, mz),
    and the sum over mz by numpy's inverse real FFT along z (which keeps the
    real part of the mz = 0 and N/2 terms, as the header's sum does).
    ``modes`` may be complex64; each plane is widened to complex128."""
    N = modes.shape[0]
    kx, ky, kz = wavenumbers(N, L)
    sx = np.asarray(sx, np.int64)
    sy = np.asarray(sy, np.int64)
    n_idx = np.arange(N)
    ey = np.exp(2j * np.pi * np.outer(sy, n_idx) / N)  # [s, my]
    Cb = np.zeros((len(sx), N // 2 + 1), np.complex128)
    Cv = np.zeros_like(Cb)
    ky2kz2 = ky[:, None] ** 2 + kz[None, :] ** 2
    for a in range(N):
        k2 = kx[a] ** 2 + ky2kz2
        A = amp * np.sqrt(power_at(np.sqrt(k2), pk, dk))
        filt = 1.0 / (1.0 + k2 / (k_F * k_F)) if np.isfinite(k_F) else 1.0
        with np.errstate(divide="ignore", invalid="ignore"):
            vf = np.where(k2 > 0, E_plus * kz[None, :] / k2, 0.0)
        g = np.asarray(modes[a], np.complex128)
        ex = np.exp(2j * np.pi * a * sx / N)[:, None]  # [s, 1]
        Cb += ex * (ey @ (A * filt * g))
        Cv += ex * (ey @ (1j * A * vf * g))
    return np.fft.irfft(Cb, n=N, axis=1) / N ** 2, np.fft.irfft(Cv, n=N, axis=1) / N ** 2
