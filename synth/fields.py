"""Seeded synthetic skewer inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the optical-depth method: it only draws the
input fields (overdensity Delta, peculiar velocity v, per-skewer pixel width,
T0, gamma) and names the workload constants.  Both the FP64 oracle and the HIP
library read its output; neither is imported here.

Field recipe (pixel units, numpy ``Generator(PCG64(seed))``):

* ``g``: a 1D Gaussian random field per skewer with power spectrum
  P(k) ~ k^-1.5 for 0 < k <= 2 pi / (10 px) and zero above (sharp cutoff);
  the k = 0 mode is zero.  White noise z ~ N(0, 1) per pixel, multiplied by
  sqrt(P(k)) in Fourier space.  ``g`` is then scaled to unit sample variance
  over the whole configuration.
* ``ln Delta = sigma * g - sigma^2 / 2``, then ``Delta /= mean(Delta)`` over the
  configuration, so that <Delta> = 1.
* ``v``: correlated with the same field as in linear theory (the 1D analogue
  of v(k) ~ i k / k^2 delta(k)): v(k) = i g(k) / k, scaled to a sample standard
  deviation of 30 km/s over the configuration.

The Gpc-scale shapes stand in for the paper's simulation boxes (4096-pixel
sight-lines through a 4096^3 grid, 20,000-spectrum sets), whose rank-ordered
density fields need a calibration hydrodynamical snapshot that is not
available.  Fields are returned as float32, skewer-major, pixel fastest.
"""
from __future__ import annotations

import dataclasses

import numpy as np

K_CUT_PIX = 10.0  # cutoff wavelength of the field, in pixels
PK_SLOPE = -1.5
SIGMA_V = 30.0  # km/s


@dataclasses.dataclass
class Workload:
    name: str
    delta: np.ndarray      # float32 [P]
    vpec: np.ndarray       # float32 [P], km/s
    offsets: np.ndarray    # int64 [S+1]
    dv: np.ndarray         # float32 [S], km/s per pixel
    T0: np.ndarray         # float32 [S], K
    gamma: np.ndarray      # float32 [S]
    target_F: float
    window_k: float
    tau_ref: float = 1.0
    delta_pivot: float = 10.0

    @property
    def n_skewers(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_pix(self) -> int:
        return int(self.offsets[-1])

    def subset(self, skewers) -> "Workload":
        """Workload made of the listed skewers (same parameters)."""
        idx = np.asarray(skewers, dtype=np.int64)
        lens = self.offsets[idx + 1] - self.offsets[idx]
        off = np.zeros(len(idx) + 1, np.int64)
        off[1:] = np.cumsum(lens)
        sel = np.concatenate([np.arange(self.offsets[s], self.offsets[s + 1])
                              for s in idx]) if len(idx) else np.zeros(0, np.int64)
        return dataclasses.replace(
            self, name=f"{self.name}[subset {len(idx)}]",
            delta=np.ascontiguousarray(self.delta[sel]),
            vpec=np.ascontiguousarray(self.vpec[sel]), offsets=off,
            dv=self.dv[idx].copy(), T0=self.T0[idx].copy(),
            gamma=self.gamma[idx].copy())


def _spectral_filters(n: int):
    """sqrt(P(k)) and the velocity filter i/k on the rfft grid of length n."""
    k = 2.0 * np.pi * np.fft.rfftfreq(n)  # radians per pixel
    amp = np.zeros_like(k)
    keep = (k > 0) & (k <= 2.0 * np.pi / K_CUT_PIX)
    amp[keep] = k[keep] ** (PK_SLOPE / 2.0)
    vfilt = np.zeros(k.shape, np.complex128)
    vfilt[keep] = 1j / k[keep]
    return amp, vfilt


def gaussian_skewers(rng: np.random.Generator, lengths):
    """Unnormalised (g, v) fields for skewers of the given lengths, drawn in
    skewer order.  Returns two float64 arrays of size sum(lengths)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    P = int(lengths.sum())
    g = np.empty(P)
    v = np.empty(P)
    uniq = np.unique(lengths)
    if len(uniq) == 1 and len(lengths) > 0 and uniq[0] > 0:
        n = int(uniq[0])
        z = rng.standard_normal((len(lengths), n))
        amp, vf = _spectral_filters(n)
        zk = np.fft.rfft(z, axis=1) * amp
        g[:] = np.fft.irfft(zk, n=n, axis=1).ravel()
        v[:] = np.fft.irfft(zk * vf, n=n, axis=1).ravel()
        return g, v
    filt = {int(n): _spectral_filters(int(n)) for n in uniq if n > 0}
    pos = 0
    for n in lengths:
        n = int(n)
        if n == 0:  # an empty skewer draws nothing
            continue
        z = rng.standard_normal(n)
        amp, vf = filt[n]
        zk = np.fft.rfft(z) * amp
        g[pos:pos + n] = np.fft.irfft(zk, n=n)
        v[pos:pos + n] = np.fft.irfft(zk * vf, n=n)
        pos += n
    return g, v


def lognormal_fields(g: np.ndarray, v: np.ndarray, sigma_lnD: float,
                     sigma_v: float = SIGMA_V):
    """Normalise (g, v) over the configuration and exponentiate g."""
    if g.size == 0:
        return np.zeros(0, np.float32), np.zeros(0, np.float32)
    if g.std() > 0:  # a 1-pixel skewer has no k > 0 mode: uniform field
        g = g / g.std()
    lnD = sigma_lnD * g - 0.5 * sigma_lnD ** 2
    D = np.exp(lnD)
    D /= D.mean()
    vs = v * (sigma_v / v.std()) if v.std() > 0 else v
    return D.astype(np.float32), vs.astype(np.float32)


def lognormal_skewers(lengths, sigma_lnD: float, seed: int,
                      rng: np.random.Generator | None = None):
    rng = rng if rng is not None else np.random.Generator(np.random.PCG64(seed))
    g, v = gaussian_skewers(rng, lengths)
    return lognormal_fields(g, v, sigma_lnD)


def _offsets(lengths):
    off = np.zeros(len(lengths) + 1, np.int64)
    off[1:] = np.cumsum(lengths)
    return off


def uniform_workload(name, n_skewers, n_pix, dv, sigma_lnD, T0, gamma,
                     target_F, window_k, seed, tau_ref=1.0, delta_pivot=10.0):
    lengths = np.full(n_skewers, n_pix, np.int64)
    D, v = lognormal_skewers(lengths, sigma_lnD, seed)
    S = n_skewers
    return Workload(name, D, v, _offsets(lengths),
                    np.full(S, dv, np.float32), np.full(S, T0, np.float32),
                    np.full(S, gamma, np.float32), target_F, window_k,
                    tau_ref, delta_pivot)


def ragged_workload(name, n_skewers, len_lo, len_hi, dv_lo, dv_hi, T0_lo,
                    T0_hi, gamma_lo, gamma_hi, sigma_lnD, target_F, window_k,
                    seed, tau_ref=1.0, delta_pivot=10.0):
    """Skewers of uneven length.  Draw order: lengths, dv, T0, gamma (each a
    vector over skewers), then the fields skewer by skewer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lengths = rng.integers(len_lo, len_hi + 1, size=n_skewers).astype(np.int64)
    dv = rng.uniform(dv_lo, dv_hi, n_skewers).astype(np.float32)
    T0 = rng.uniform(T0_lo, T0_hi, n_skewers).astype(np.float32)
    gamma = rng.uniform(gamma_lo, gamma_hi, n_skewers).astype(np.float32)
    D, v = lognormal_skewers(lengths, sigma_lnD, seed, rng=rng)
    return Workload(name, D, v, _offsets(lengths), dv, T0, gamma, target_F,
                    window_k, tau_ref, delta_pivot)


# --------------------------------------------------------------------------
# The five workloads.  "C1 statistics" = sigma_lnD 1.0, dv 2 km/s,
# T0 1.5e4 K, gamma 1.5, target mean flux 0.8.

def config1(seed: int = 1) -> Workload:
    """64 skewers x 1024 px, dv 2 km/s (box 2048 km/s), sigma_lnD 1.0,
    T0 1.5e4 K, gamma 1.5, target <F> 0.8; full-sum reference."""
    return uniform_workload("C1 64x1024", 64, 1024, 2.0, 1.0, 1.5e4, 1.5, 0.8,
                            6.0, seed)


def config2(seed: int = 2) -> Workload:
    """4096 skewers x 4096 px, dv 2 km/s, sigma_lnD 1.2, T0 2e4 K, gamma 1.3,
    target <F> 0.75, window +-6 b."""
    return uniform_workload("C2 4096x4096", 4096, 4096, 2.0, 1.2, 2.0e4, 1.3,
                            0.75, 6.0, seed)


def config3(seed: int = 3, n_skewers: int = 20000) -> Workload:
    """20000 skewers, lengths uniform in [512, 8192] px, dv uniform in [1, 4]
    km/s, T0 uniform in [1e4, 2.5e4] K, gamma uniform in [1.1, 1.6];
    sigma_lnD 1.0 and target <F> 0.8 (C1 statistics)."""
    return ragged_workload(f"C3 ragged {n_skewers}", n_skewers, 512, 8192,
                           1.0, 4.0, 1.0e4, 2.5e4, 1.1, 1.6, 1.0, 0.8, 6.0,
                           seed)


def config5(seed: int = 5) -> Workload:
    """4096 skewers x 2048 px with C1 statistics (adjoint workload)."""
    return uniform_workload("C5 4096x2048", 4096, 2048, 2.0, 1.0, 1.5e4, 1.5,
                            0.8, 6.0, seed)


def gpc_lowres(seed: int = 6, n_skewers: int = 4096) -> Workload:
    """Sight-lines through a 1 Gpc, 4096^3 box at z = 3 (Section 3.2): 4096 px
    of ~244 comoving kpc, i.e. dv = 18.3 km/s at H(z=3) = 300.2 km/s/Mpc;
    T0 = 1.7e4 K, gamma = 1.3 (Section 3), target <F> = 0.72 (Section 2.3),
    C1 field statistics."""
    return uniform_workload(f"Gpc {n_skewers}x4096", n_skewers, 4096, 18.3, 1.0, 1.7e4, 1.3,
                            0.72, 6.0, seed)


# Instrument settings as the paper prints them (widths in km/s or Angstrom;
# Angstrom widths are converted at the model redshift by whoever uses them).
REDSHIFT = 3.0
INSTRUMENT_HIGH_RES = dict(fwhm_kms=7.0, bin_angstrom=0.05, snr=50.0)  # Section 3.1
INSTRUMENT_BOSS = dict(fwhm_angstrom=3.63, bin_angstrom=1.0375, snr=5.0,
                       proximity_kms=3000.0)  # Section 3.2
INSTRUMENT_SDSS = dict(fwhm_kms=170.0, bin_angstrom=1.0, snr=3.8)  # Section 4.2


def synthetic_flux(lengths, seed: int, tau_mean: float = 0.35, sigma: float = 1.2) -> np.ndarray:
    """A flux field F = exp(-tau) with a lognormal optical depth of the given
    mean, drawn from the same Gaussian random field recipe as Delta (float32,
    skewer-major).  It stands in for a forward flux where a stage downstream of
    F is tested on its own."""
    D, _ = lognormal_skewers(np.asarray(lengths, np.int64), sigma, seed)
    return np.exp(-tau_mean * D.astype(np.float64)).astype(np.float32)


def noise_draws(n: int, seed: int) -> np.ndarray:
    """Standard-normal draws for the additive noise, float32 [n]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(n).astype(np.float32)


def small_workload(n_skewers=8, n_pix=256, seed=11, sigma_lnD=1.0, dv=2.0,
                   T0=1.5e4, gamma=1.5, target_F=0.8, window_k=6.0):
    return uniform_workload(f"small {n_skewers}x{n_pix}", n_skewers, n_pix, dv,
                            sigma_lnD, T0, gamma, target_F, window_k, seed)


def lognormal_box_3d(nx: int, ny: int, nz: int, sigma_lnD: float, seed: int,
                     device="cpu", sigma_v: float = SIGMA_V):
    """3D lognormal field of nx*ny skewers of nz pixels (skewer axis z,
    contiguous), 3D P(k) ~ k^-1.5 with a sharp cutoff at 2 pi / (10 px), the
    velocity along z from v(k) = i k_z / k^2 g(k), generated with torch.fft on
    ``device`` (a seeded torch.Generator draws the white noise).  Returns
    float32 torch tensors (Delta, v) of shape [nx*ny*nz]."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    z = torch.randn((nx, ny, nz), generator=gen, device=device,
                    dtype=torch.float32)
    zk = torch.fft.rfftn(z)
    del z
    kx = 2 * np.pi * torch.fft.fftfreq(nx, device=device)
    ky = 2 * np.pi * torch.fft.fftfreq(ny, device=device)
    kz = 2 * np.pi * torch.fft.rfftfreq(nz, device=device)
    k2 = (kx[:, None, None] ** 2 + ky[None, :, None] ** 2
          + kz[None, None, :] ** 2)
    kmag = torch.sqrt(k2)
    keep = (kmag > 0) & (kmag <= 2 * np.pi / K_CUT_PIX)
    amp = torch.where(keep, kmag.clamp_min(1e-30) ** (PK_SLOPE / 2.0),
                      torch.zeros_like(kmag))
    del kmag
    zk *= amp
    del amp
    vf = torch.where(keep, kz[None, None, :] / k2.clamp_min(1e-30),
                     torch.zeros_like(k2))
    del k2, keep
    vk = zk * (1j * vf)
    del vf
    g = torch.fft.irfftn(zk, s=(nx, ny, nz))
    del zk
    v = torch.fft.irfftn(vk, s=(nx, ny, nz))
    del vk
    g = g / g.double().std().float()
    lnD = sigma_lnD * g - 0.5 * sigma_lnD ** 2
    del g
    D = torch.exp(lnD)
    del lnD
    D = D / D.double().mean().float()
    v = v * (sigma_v / v.double().std().float())
    return D.reshape(-1).contiguous(), v.reshape(-1).contiguous()


def config4(seed: int = 4, nx: int = 512, ny: int = 512, nz: int = 4096,
            device="cpu") -> Workload:
    """512 x 512 skewers of 4096 px through one seeded 3D lognormal field
    (C1 statistics); arrays stay torch tensors on ``device``."""
    D, v = lognormal_box_3d(nx, ny, nz, 1.0, seed, device=device)
    S = nx * ny
    lengths = np.full(S, nz, np.int64)
    return Workload(f"C4 box {nx}x{ny}x{nz}", D, v, _offsets(lengths),
                    np.full(S, 2.0, np.float32), np.full(S, 1.5e4, np.float32),
                    np.full(S, 1.5, np.float32), 0.8, 6.0)


# ---------------------------------------------------------------------------
# Inputs of the skewer-only field synthesis (Section 2.1, eqs. 1 and 3).

# Cosmology of the paper's calibration run (Section 2): h, Omega_m, n_s.
H_LITTLE, OMEGA_M, N_S = 0.72, 0.26, 0.96
K_F_MPC = 6.5  # filtering wavenumber of eq. (1), Mpc^-1 (Section 2.1)
# E_+ = H(z) f / (1 + z) at z = 3 with H(3) = 300.2 km/s/Mpc and
# f = Omega_m(z)^0.55 = 0.976; the growth factor is folded into the amplitude.
E_PLUS_Z3 = 300.2 * 0.976 / 4.0


@dataclasses.dataclass
class FieldInputs:
    name: str
    n: int                 # grid points per side
    modes: object          # complex64 [n, n, n/2+1] (numpy, or a torch tensor)
    pk: np.ndarray         # float64 [n_table]: P at |k| = j dk
    dk: float              # Mpc^-1
    amp: float
    box: float             # Mpc
    k_F: float             # Mpc^-1
    E_plus: float          # km/s Mpc
    sx: np.ndarray         # int32 [S]
    sy: np.ndarray         # int32 [S]


def bbks_power_table(n: int, box: float, n_table: int = 4096):
    """Linear power shape P(k) = k^n_s T(q)^2 with the BBKS transfer function,
    T(q) = ln(1 + 2.34 q) / (2.34 q) [1 + 3.89 q + (16.1 q)^2 + (5.46 q)^3 +
    (6.71 q)^4]^(-1/4), q = k / (Omega_m h^2) (k in Mpc^-1): a closed-form
    stand-in for the Eisenstein & Hu transfer function the paper uses, which is
    not available here.  Tabulated at j dk up to just past the grid's largest
    |k| = sqrt(3) pi n / box.  Returns (table float64 [n_table], dk)."""
    kmax = np.sqrt(3.0) * np.pi * n / box
    dk = kmax * 1.001 / (n_table - 1)
    k = np.arange(n_table) * dk
    q = k / (OMEGA_M * H_LITTLE ** 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        T = np.where(q > 0, np.log1p(2.34 * q) / (2.34 * q), 1.0) * (
            1 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4) ** -0.25
    return (k ** N_S * T ** 2).astype(np.float64), float(dk)


def _unit_rms_amp(n, box, pk, dk):
    """Amplitude that gives delta_DM unit variance for modes of E|g|^2 = n^3
    (the transform of unit white noise): Var = n^-3 sum over the full spectrum
    of amp^2 P(|k|), counted on the half-spectrum with weight 2 for 0 < mz < n/2."""
    m = np.fft.fftfreq(n, d=1.0 / n)
    mz = np.arange(n // 2 + 1, dtype=np.float64)
    w = np.where((mz == 0) | (mz == n // 2), 1.0, 2.0)
    f = 2 * np.pi / box
    tot = 0.0
    for a in m:
        k = f * np.sqrt(a * a + m[:, None] ** 2 + mz[None, :] ** 2)
        tot += float(np.sum(w[None, :] * np.interp(k, np.arange(pk.size) * dk, pk, right=0.0)))
    return 1.0 / np.sqrt(tot / n ** 3)


def field_columns(n: int, n_lines: int, seed: int):
    """n_lines distinct random columns (sx, sy) of an n x n grid, int32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.choice(n * n, size=n_lines, replace=False)
    return (c // n).astype(np.int32), (c % n).astype(np.int32)


def field_modes_white(n: int, seed: int, device="cpu"):
    """The half-spectrum of unit-variance real white noise on an n^3 grid
    (torch.fft.rfftn of seeded torch normals): complex64 torch tensor
    [n, n, n/2+1] on ``device``, E|g|^2 = n^3, Hermitian where a real field's
    spectrum is."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    z = torch.randn((n, n, n), generator=gen, device=device, dtype=torch.float32)
    g = torch.fft.rfftn(z)
    del z
    return g.to(torch.complex64).contiguous()


def field_synthesis_workload(n: int = 1024, n_lines: int = 6250, seed: int = 7,
                             device="cpu") -> FieldInputs:
    """Sight-lines through a box of the paper's Gpc-run cell size (1 Gpc /
    4096 = 0.244 Mpc, so 250 Mpc at n = 1024), at the paper's sight-line
    density (100,000 per 4096^2 columns: 6,250 per 1024^2), k_F = 6.5 Mpc^-1,
    E_+ at z = 3, the BBKS power shape scaled to unit rms delta_DM, modes from
    real white noise (generated with torch on ``device``)."""
    box = n * 1000.0 / 4096.0
    pk, dk = bbks_power_table(n, box)
    amp = _unit_rms_amp(n, box, pk, dk)
    sx, sy = field_columns(n, n_lines, seed)
    return FieldInputs(f"field synthesis {n}^3, {n_lines} sight-lines", n,
                       field_modes_white(n, seed, device), pk, dk, amp, box, K_F_MPC,
                       E_PLUS_Z3, sx, sy)


# ---------------------------------------------------------------------------
# Inputs of the 3D flux power spectrum reconstruction (Section 6.2, eq. 7).

@dataclasses.dataclass
class Power3dInputs:
    name: str
    n: int                 # grid points per side = pixels per sight-line
    box: float             # Mpc
    F: np.ndarray          # float32 [S * n], sight-line-major
    mean_F: float
    p_noise: float         # flat 1D noise power, Mpc
    sx: np.ndarray         # int32 [S]
    sy: np.ndarray         # int32 [S]


def power3d_workload(n: int = 1024, n_lines: int = 6250, seed: int = 8,
                     snr: float = 5.0) -> Power3dInputs:
    """A mock survey in a box of the paper's Gpc-run cell size (250 Mpc at
    n = 1024) at its sight-line density (6,250 distinct columns of 1024^2):
    synthetic flux (lognormal optical depth, mean 0.35) on every sight-line,
    the mean flux of the sample as Fbar, and the flat noise power of S/N = 5
    per pixel, (1 / (S/N Fbar))^2 L / n."""
    box = n * 1000.0 / 4096.0
    F = synthetic_flux(np.full(n_lines, n, np.int64), seed)
    mean_F = float(np.mean(F, dtype=np.float64))
    sx, sy = field_columns(n, n_lines, seed)
    p_noise = (1.0 / (snr * mean_F)) ** 2 * box / n
    return Power3dInputs(f"3D flux power {n}^3, {n_lines} sight-lines", n, box, F, mean_F,
                         p_noise, sx, sy)
