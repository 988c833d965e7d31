"""Pins of the field-synthesis oracle (oracle/field_synthesis.py) against
what the paper's definitions and the mathematics fix, independently of numpy's
inverse FFT: the explicit sum over the half-spectrum, single-mode closed forms
of eq. (1) and eq. (3), Parseval's identity, the filter's limit and the power
table's interpolation.  CPU only."""
import math

import numpy as np
import pytest

from oracle import field_synthesis as FS


def _random_modes(N, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(N, N, N // 2 + 1)) + 1j * rng.normal(size=(N, N, N // 2 + 1))


def _table(n=64, dk=0.25, seed=3):
    rng = np.random.default_rng(seed)
    return np.abs(rng.normal(1.0, 0.3, n)), dk


@pytest.mark.parametrize("N", [4, 6])
def test_matches_the_explicit_sum_on_small_grids(N):
    """The real-field map is the sum over the half-spectrum with weights 1 on
    the kz = 0 and N/2 planes and 2 elsewhere (brute force, no FFT)."""
    modes = _random_modes(N, N)
    pk, dk = _table()
    L, kF, Ep = 7.0, 3.0, 50.0
    sx, sy = np.repeat(np.arange(N), N), np.tile(np.arange(N), N)
    fb, fv = FS.skewer_fields(modes, pk, dk, 0.7, L, kF, Ep, sx, sy)
    db, vk = FS.spectra(modes, pk, dk, 0.7, L, kF, Ep)
    for s in range(0, N * N, 3):
        for z in range(N):
            assert abs(fb[s, z] - FS.explicit_sum(db, sx[s], sy[s], z)) <= 1e-13
            assert abs(fv[s, z] - FS.explicit_sum(vk, sx[s], sy[s], z)) <= 1e-11


@pytest.mark.parametrize("mode", [(3, 13, 5), (1, 0, 0), (2, 5, 8), (0, 0, 1)])
def test_single_mode_closed_forms(mode):
    """One mode g at n = (a, b, c): delta_b = (w/N^3) A/(1 + k^2/k_F^2) |g|
    cos(theta + arg g) and v_z = -(w/N^3) E_+ A (k_z/k^2) |g| sin(theta + arg g),
    A = amp sqrt(P(|k|)), theta = 2 pi (a x + b y + c z)/N, w = 2 for
    0 < c < N/2 else 1 (eq. 1, eq. 3)."""
    N, L, kF, Ep, amp = 16, 12.0, 2.5, 80.0, 3.0
    a, b, c = mode
    g = 0.6 - 1.1j
    modes = np.zeros((N, N, N // 2 + 1), complex)
    modes[a, b, c] = g
    pk, dk = _table(n=40, dk=0.3)
    sx, sy = np.repeat(np.arange(N), N), np.tile(np.arange(N), N)
    fb, fv = FS.skewer_fields(modes, pk, dk, amp, L, kF, Ep, sx, sy)
    na = a - N if a > N // 2 else a
    nb = b - N if b > N // 2 else b
    kvec = 2 * math.pi / L * np.array([na, nb, c], float)
    k2 = float(kvec @ kvec)
    A = amp * math.sqrt(np.interp(math.sqrt(k2), np.arange(40) * dk, pk))
    w = 2.0 if 0 < c < N // 2 else 1.0
    z = np.arange(N)
    for s in range(N * N):
        th = 2 * math.pi * (a * sx[s] + b * sy[s] + c * z) / N + np.angle(g)
        ref_b = w / N ** 3 * A / (1 + k2 / kF ** 2) * abs(g) * np.cos(th)
        ref_v = -w / N ** 3 * Ep * A * (kvec[2] / k2) * abs(g) * np.sin(th)
        np.testing.assert_allclose(fb[s], ref_b, rtol=0, atol=1e-12 * abs(ref_b).max() + 1e-300)
        np.testing.assert_allclose(fv[s], ref_v, rtol=0, atol=1e-12 * max(abs(ref_v).max(), 1e-300))


def test_parseval():
    """Modes only on 0 < kz < N/2: sum over the box of f^2 = (2/N^3) sum |F|^2."""
    N = 16
    modes = _random_modes(N, 5)
    modes[:, :, 0] = 0
    modes[:, :, N // 2] = 0
    pk, dk = _table()
    sx, sy = np.repeat(np.arange(N), N), np.tile(np.arange(N), N)
    fb, fv = FS.skewer_fields(modes, pk, dk, 1.0, 9.0, 4.0, 30.0, sx, sy)
    db, vk = FS.spectra(modes, pk, dk, 1.0, 9.0, 4.0, 30.0)
    assert abs((fb ** 2).sum() / (2 / N ** 3 * (abs(db) ** 2).sum()) - 1) < 1e-12
    assert abs((fv ** 2).sum() / (2 / N ** 3 * (abs(vk) ** 2).sum()) - 1) < 1e-12


def test_filter_limit_and_ratio():
    """k_F -> infinity leaves the dark-matter field; a finite k_F scales each
    mode by 1/(1 + k^2/k_F^2) (eq. 1)."""
    N = 8
    modes = _random_modes(N, 6)
    pk, dk = _table()
    sx, sy = np.arange(N), (3 * np.arange(N)) % N
    f_inf, _ = FS.skewer_fields(modes, pk, dk, 1.0, 5.0, math.inf, 10.0, sx, sy)
    dm = FS.real_field(1.0 * np.sqrt(FS.power_at(
        np.sqrt(sum(np.meshgrid(*[k ** 2 for k in FS.wavenumbers(N, 5.0)], indexing="ij"))),
        pk, dk)) * modes)
    np.testing.assert_allclose(f_inf, dm[sx, sy, :], rtol=0, atol=1e-14)
    db_f, _ = FS.spectra(modes, pk, dk, 1.0, 5.0, 1.7, 10.0)
    db_i, _ = FS.spectra(modes, pk, dk, 1.0, 5.0, math.inf, 10.0)
    kx, ky, kz = FS.wavenumbers(N, 5.0)
    k2 = kx[:, None, None] ** 2 + ky[None, :, None] ** 2 + kz[None, None, :] ** 2
    np.testing.assert_allclose(db_f, db_i / (1 + k2 / 1.7 ** 2), rtol=1e-15, atol=0)


def test_velocity_ratio_and_zero_mode():
    """v_z(k) / delta_DM(k) = i E_+ k_z / k^2 for every k != 0 (eq. 3), and the
    k = 0 mode carries no velocity."""
    N = 8
    modes = _random_modes(N, 7)
    pk, dk = _table()
    db, vk = FS.spectra(modes, pk, dk, 2.0, 6.0, math.inf, 25.0)
    kx, ky, kz = FS.wavenumbers(N, 6.0)
    k2 = kx[:, None, None] ** 2 + ky[None, :, None] ** 2 + kz[None, None, :] ** 2
    nz = k2 > 0
    np.testing.assert_allclose(vk[nz], (1j * 25.0 * (kz[None, None, :] / np.where(nz, k2, 1))
                                        * db)[nz], rtol=1e-15)
    assert vk[0, 0, 0] == 0


def test_power_table_interpolation_is_exact_for_a_linear_table():
    dk = 0.1
    j = np.arange(100) * dk
    pk = 2.0 + 3.0 * j
    k = np.array([0.0, 0.05, 1.234, 9.89])
    np.testing.assert_allclose(FS.power_at(k, pk, dk), 2.0 + 3.0 * k, rtol=1e-15)
    assert FS.power_at(np.array([10.0, 50.0]), pk, dk)[1] == 0.0


def test_direct_sight_line_path_matches_the_grid_path():
    """The per-sight-line direct sums (used at full size) agree with the
    full-grid inverse transform."""
    N = 32
    modes = _random_modes(N, 9)
    pk, dk = _table(n=80, dk=0.1)
    rng = np.random.default_rng(4)
    sx, sy = rng.integers(0, N, 40), rng.integers(0, N, 40)
    a = FS.skewer_fields(modes, pk, dk, 1.5, 20.0, 2.0, 60.0, sx, sy)
    b = FS.skewer_fields_direct(modes, pk, dk, 1.5, 20.0, 2.0, 60.0, sx, sy)
    for f, g in zip(a, b):
        assert np.abs(f - g).max() <= 1e-12 * np.abs(f).max()


@pytest.mark.parametrize("N,kF", [(8, 3.0), (16, np.inf)])
def test_plane_by_plane_path_matches_the_grid_path(N, kF):
    """The memory-light path (one mx plane at a time, complex64 input widened
    per plane) gives the grid path's values on chosen sight-lines, including
    repeated and shared-row columns."""
    modes = _random_modes(N, 7 + N).astype(np.complex64)
    pk, dk = _table(n=80, dk=0.2)
    L, Ep, amp = 9.0, 60.0, 1.3
    sx = np.array([0, 3, N - 1, 5, 5, 2])
    sy = np.array([0, 3, 1, 1, 1, N - 1])
    fb, fv = FS.skewer_fields(modes.astype(np.complex128), pk, dk, amp, L, kF, Ep, sx, sy)
    pb, pv = FS.skewer_fields_planes(modes, pk, dk, amp, L, kF, Ep, sx, sy)
    assert np.max(np.abs(pb - fb)) <= 1e-13 * np.max(np.abs(fb))
    assert np.max(np.abs(pv - fv)) <= 1e-13 * np.max(np.abs(fv))
