"""Pins of the 3D flux power oracle (oracle/flux_power_3d.py, eq. 7 of
Section 6.2) against brute-force sums and closed forms.  CPU only."""
import math

import numpy as np
import pytest

from oracle import flux_power_3d as P3


def _survey(n, S, seed):
    rng = np.random.default_rng(seed)
    sx, sy = rng.integers(0, n, S), rng.integers(0, n, S)
    F = np.exp(-np.exp(rng.normal(-1.0, 1.0, (S, n))))
    return F.ravel(), sx, sy


@pytest.mark.parametrize("n,S", [(4, 5), (6, 9)])
def test_box_power_against_brute_force_dft(n, S):
    F, sx, sy = _survey(n, S, n)
    sx[1], sy[1] = sx[0], sy[0]  # two sight-lines in one column
    L, mean_F = 3.0, 0.7
    w = np.linspace(0.5, 1.5, S)
    P_true, P_box, P_1d, P_2d = P3.reconstruct(F, mean_F, sx, sy, n, L, w, p_noise=0.01)
    d = (F.reshape(S, n) / mean_F - 1.0)
    for kx in range(n):
        for ky in range(n):
            W = sum(w[s] * np.exp(-2j * math.pi * (kx * sx[s] + ky * sy[s]) / n) for s in range(S))
            assert abs(P_2d[kx, ky] - L ** 2 / n ** 4 * abs(W) ** 2) <= 1e-12 * (1 + P_2d[kx, ky])
            for kz in range(n // 2 + 1):
                D = 0j
                for s in range(S):
                    for z in range(n):
                        D += w[s] * d[s, z] * np.exp(-2j * math.pi * (kx * sx[s] + ky * sy[s]
                                                                      + kz * z) / n)
                assert abs(P_box[kx, ky, kz] - L ** 3 / n ** 6 * abs(D) ** 2) <= 1e-12 * (
                    1 + P_box[kx, ky, kz])
    for kz in range(n // 2 + 1):
        g = [abs(sum(d[s, z] * np.exp(-2j * math.pi * kz * z / n) for z in range(n))) ** 2
             for s in range(S)]
        assert abs(P_1d[kz] - L / n ** 2 * np.mean(g)) <= 1e-12 * (1 + P_1d[kz])
    np.testing.assert_allclose(P_true, P_box - (P_1d[None, None, :] + 0.01) * P_2d[:, :, None],
                               rtol=0, atol=1e-15 * np.abs(P_box).max())


def test_identical_sight_lines_have_no_true_power():
    """Every sight-line carrying the same spectrum: the box's power is all
    aliasing, P_box = P_1D P_2D,w, so P_true = 0 for every mode."""
    n, S = 16, 12
    rng = np.random.default_rng(1)
    one = np.exp(-np.exp(rng.normal(-1, 1, n)))
    F = np.tile(one, S)
    sx, sy = rng.permutation(n * n)[:S] // n, rng.permutation(n * n)[:S] % n
    P_true, P_box, _, _ = P3.reconstruct(F, 0.8, sx, sy, n, 50.0)
    assert np.abs(P_true).max() <= 1e-12 * np.abs(P_box).max()


def test_single_sight_line_leaves_minus_the_noise_term():
    """S = 1: P_box = P_1D (L^2/n^4), so P_true = -P_N L^2 / n^4 everywhere."""
    n, L, pn = 8, 20.0, 0.3
    F, sx, sy = _survey(n, 1, 2)
    P_true, P_box, _, P_2d = P3.reconstruct(F, 0.6, sx, sy, n, L, p_noise=pn)
    np.testing.assert_allclose(P_2d, L ** 2 / n ** 4, rtol=1e-14)
    np.testing.assert_allclose(P_true, -pn * L ** 2 / n ** 4, rtol=0,
                               atol=1e-12 * np.abs(P_box).max())


def test_parseval_of_the_box():
    """Sum over all modes of |D|^2 (conjugate partners counted) = n^3 times the
    sum of the squared box (distinct columns)."""
    n, S = 16, 20
    F, _, _ = _survey(n, S, 3)
    cols = np.random.default_rng(3).permutation(n * n)[:S]
    sx, sy = cols // n, cols % n
    _, P_box, _, _ = P3.reconstruct(F, 0.75, sx, sy, n, 1.0)
    c = np.where((np.arange(n // 2 + 1) == 0) | (np.arange(n // 2 + 1) == n // 2), 1.0, 2.0)
    total = (P_box * c[None, None, :]).sum() * n ** 6
    box = ((F.reshape(S, n) / 0.75 - 1.0) ** 2).sum()
    assert abs(total / (n ** 3 * box) - 1) < 1e-12


def test_shell_counts_and_mean_k_by_brute_force():
    n, L, nb = 8, 10.0, 9
    P = np.ones((n, n, n // 2 + 1))
    cnt, kmean, pt, pb = P3.shell_average(P, 2 * P, n, L, nb)
    want = np.zeros(nb)
    ksum = np.zeros(nb)
    for a in range(n):
        for b in range(n):
            for c in range(n):  # the full lattice
                m = [(v + n // 2) % n - n // 2 for v in (a, b, c)]
                # the half-spectrum keeps mz = 0 .. n/2; mz = -n/2 is mz = n/2
                r = math.sqrt(sum(v * v for v in m))
                if int(r) < nb:
                    want[int(r)] += 1
                    ksum[int(r)] += r
    np.testing.assert_allclose(cnt, want)
    np.testing.assert_allclose(kmean, np.where(want > 0, ksum / np.maximum(want, 1), 0)
                               * 2 * math.pi / L, rtol=1e-14)
    np.testing.assert_allclose(pt[cnt > 0], 1.0)
    np.testing.assert_allclose(pb[cnt > 0], 2.0)


def test_noise_term_is_linear():
    n, S = 8, 6
    F, sx, sy = _survey(n, S, 5)
    a = P3.flux_power_3d(F, 0.7, sx, sy, n, 5.0, 8, p_noise=0.0)[2]
    b = P3.flux_power_3d(F, 0.7, sx, sy, n, 5.0, 8, p_noise=0.5)[2]
    c = P3.flux_power_3d(F, 0.7, sx, sy, n, 5.0, 8, p_noise=1.0)[2]
    np.testing.assert_allclose(c - a, 2 * (b - a), rtol=1e-12, atol=1e-15)
