"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

None of these checks re-evaluates the oracle's own double sum: each compares it
with a closed form (Poisson-summed lattice of Gaussians = Jacobi theta function,
Gaussian moments), an invariance of eq. (6), a printed value of the paper, a
library routine, or a 40-digit brute force over the full image lattice.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest

from oracle import oracle as O
from synth import fields

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Physical constants as quoted in CGS tables; the oracle defines its own.
KB = 1.380649e-16
MH = 1.6735575e-24


def b_of_T(T):
    return math.sqrt(2 * KB * T / MH) / 1e5


def theta3(v, dv, b):
    """Poisson summation of the unit-spaced lattice of Gaussians:
    (dv / (sqrt(pi) b)) sum_m exp(-((m dv - v)/b)^2) = theta_3(pi v / dv, q),
    q = exp(-pi^2 b^2 / dv^2)."""
    q = mpmath.exp(-(mpmath.pi ** 2) * mpmath.mpf(b) ** 2 / mpmath.mpf(dv) ** 2)
    return float(mpmath.jtheta(3, mpmath.pi * mpmath.mpf(v) / dv, q))


def run_tau(delta, v, dv, T0, gamma, S=1, **kw):
    return O.tau(np.asarray(delta, float), np.asarray(v, float), dv, T0, gamma,
                 n_skewers=S, **kw)


# --------------------------------------------------------------------------
def test_doppler_parameter_textbook():
    g = json.load(open(os.path.join(GOLDEN, "doppler_b.json")))
    assert abs(O.doppler_b(g["T_K"]) - g["b_kms"]) < g["abs_tol_kms"]
    # b scales as sqrt(T)
    assert O.doppler_b(4e4) == pytest.approx(2 * O.doppler_b(1e4), rel=1e-15)


@pytest.mark.parametrize("c,v0,dv,T0,gamma", [
    (1.0, 0.0, 2.0, 1.0e4, 1.5),      # the Gunn-Peterson case itself
    (1.0, 7.3, 2.0, 2.0e4, 1.3),      # bulk velocity is irrelevant when resolved
    (3.0, -4.0, 2.0, 1.5e4, 1.5),     # Delta^2 and T(Delta) enter
    (0.3, 11.0, 40.0, 1.2e4, 1.6),    # b/dv = 0.3: the lattice correction is large
    (1.7, 25.0, 30.0, 1.0e4, 0.8),    # gamma < 1 (inverted relation)
])
def test_gunn_peterson_uniform_field(c, v0, dv, T0, gamma):
    """Uniform Delta = c, constant v: every pixel has
    tau = tau_ref c^2 (T/1e4)^-0.7 theta_3(pi v/dv, q) with T = T0 c^(gamma-1)."""
    N = 256  # V/2 >= 12 b: the box truncates the lattice below 1e-60
    tau_ref = 1.7
    t = run_tau(np.full(N, c), np.full(N, v0), dv, T0, gamma, tau_ref=tau_ref)
    T = T0 * c ** (gamma - 1)
    expect = tau_ref * c * c * (T / 1e4) ** -0.7 * theta3(v0, dv, b_of_T(T))
    np.testing.assert_allclose(t, expect, rtol=1e-13)
    assert np.ptp(t) <= 1e-13 * expect


def test_pivot_caps_temperature():
    """Above Delta = 10 the temperature is T(Delta = 10) (Sec. 2.3, eq. 5 pivot)."""
    N, dv, T0, gamma = 512, 2.0, 1.5e4, 1.5  # V/2 >= 12 b
    t = run_tau(np.full(N, 20.0), np.zeros(N), dv, T0, gamma)
    T = T0 * 10.0 ** (gamma - 1)
    expect = 400.0 * (T / 1e4) ** -0.7 * theta3(0.0, dv, b_of_T(T))
    np.testing.assert_allclose(t, expect, rtol=1e-13)
    # exactly at the pivot the power-law branch applies (continuity)
    t10 = run_tau(np.full(N, 10.0), np.zeros(N), dv, T0, gamma)
    np.testing.assert_allclose(t10, 100.0 * (T / 1e4) ** -0.7, rtol=1e-13)
    # disabling the pivot restores the pure power law
    t_np = run_tau(np.full(N, 20.0), np.zeros(N), dv, T0, gamma,
                   delta_pivot=math.inf)
    T2 = T0 * 20.0 ** (gamma - 1)
    np.testing.assert_allclose(t_np, 400.0 * (T2 / 1e4) ** -0.7, rtol=1e-13)


@pytest.mark.parametrize("j0,vstar_px,dv", [(5, -9, 2.0), (120, 13, 1.5), (64, 0, 3.0)])
def test_isolated_line_shape_and_position(j0, vstar_px, dv):
    """One non-empty pixel gives one Gaussian line centred at j0 + v/dv (mod N),
    symmetric about its centre, with the Gaussian's second moment b^2/(2 dv^2)
    and area tau_ref Delta^2 (T/1e4)^-0.7 (the line wraps round the box)."""
    N, T0, gamma, Dstar = 256, 1.5e4, 1.5, 2.5  # V/2 >= 9 b
    delta = np.zeros(N)
    delta[j0] = Dstar
    v = np.zeros(N)
    v[j0] = vstar_px * dv
    t = run_tau(delta, v, dv, T0, gamma)
    c = (j0 + vstar_px) % N
    assert int(np.argmax(t)) == c
    m = np.arange(1, N // 2)
    np.testing.assert_allclose(t[(c + m) % N], t[(c - m) % N], rtol=1e-12, atol=1e-300)
    T = T0 * Dstar ** (gamma - 1)
    b = b_of_T(T)
    area = t.sum()
    assert area == pytest.approx(Dstar ** 2 * (T / 1e4) ** -0.7 *
                                 theta3(vstar_px * dv, dv, b), rel=1e-13)
    off = ((np.arange(N) - c + N // 2) % N) - N // 2  # signed distance to centre
    var = (t * (off * dv) ** 2).sum() / area
    assert var == pytest.approx(b * b / 2.0, rel=1e-10)


def test_equivalent_width_with_lattice_correction():
    """Sum_i tau_i = tau_ref sum_j Delta_j^2 (T_j/1e4)^-0.7 theta_3(pi v_j/dv, q_j),
    for any Delta and v field; includes cold sources with b/dv < 1 where the
    Poisson correction is far from negligible."""
    rng = np.random.default_rng(7)
    N, dv, T0, gamma = 256, 9.0, 1.2e4, 1.4
    delta = np.exp(rng.normal(0, 1.2, N))
    delta[rng.integers(0, N, 10)] = 0.0
    v = rng.normal(0, 30, N)
    t = run_tau(delta, v, dv, T0, gamma)
    expect = 0.0
    for j in range(N):
        if delta[j] == 0:
            continue
        D = min(delta[j], 10.0)
        T = T0 * D ** (gamma - 1)
        expect += delta[j] ** 2 * (T / 1e4) ** -0.7 * theta3(v[j], dv, b_of_T(T))
    assert t.sum() == pytest.approx(expect, rel=1e-13)


def test_equivariances():
    """Cyclic shift, reflection and a bulk shift by one pixel width."""
    w = fields.small_workload(n_skewers=1, n_pix=192, seed=5)
    d, v = w.delta.astype(float), w.vpec.astype(float)
    dv, T0, gamma = 2.0, 1.5e4, 1.5
    t = run_tau(d, v, dv, T0, gamma)
    for m in (1, 17, 100):
        ts = run_tau(np.roll(d, m), np.roll(v, m), dv, T0, gamma)
        np.testing.assert_allclose(ts, np.roll(t, m), rtol=1e-12)
    tr = run_tau(d[::-1], -v[::-1], dv, T0, gamma)
    np.testing.assert_allclose(tr, t[::-1], rtol=1e-12)
    tb = run_tau(d, v + dv, dv, T0, gamma)
    np.testing.assert_allclose(tb, np.roll(t, 1), rtol=1e-12)
    t3 = run_tau(d, v, dv, T0, gamma, tau_ref=3.0)
    np.testing.assert_allclose(t3, 3.0 * t, rtol=1e-14)


def _mp_tau_lattice(delta, v, dv, T0, gamma, images=3):
    """40-digit brute force over the full periodic lattice (all images)."""
    mpmath.mp.dps = 40
    N = len(delta)
    V = mpmath.mpf(N) * dv
    out = []
    for i in range(N):
        acc = mpmath.mpf(0)
        for j in range(N):
            if delta[j] == 0:
                continue
            D = min(mpmath.mpf(delta[j]), mpmath.mpf(10))
            T = mpmath.mpf(T0) * D ** (mpmath.mpf(gamma) - 1)
            b = mpmath.sqrt(2 * mpmath.mpf(KB) * T / mpmath.mpf(MH)) / 10 ** 5
            w = (mpmath.mpf(delta[j]) ** 2 * (T / 10 ** 4) ** mpmath.mpf(-0.7)
                 * dv / (mpmath.sqrt(mpmath.pi) * b))
            for m in range(-images, images + 1):
                d = (i - j) * mpmath.mpf(dv) - mpmath.mpf(v[j]) + m * V
                acc += w * mpmath.exp(-(d / b) ** 2)
        out.append(float(acc))
    mpmath.mp.dps = 15
    return np.array(out)


@pytest.mark.parametrize("N,seed", [(1, 0), (2, 1), (3, 2), (5, 3), (8, 4), (16, 5)])
def test_brute_force_lattice(N, seed):
    """Tiny boxes with V >= 12 b: minimal image equals the lattice sum to
    exp(-36), so the 40-digit lattice sum must match to rounding."""
    rng = np.random.default_rng(seed)
    dv = 100.0
    delta = np.exp(rng.normal(0, 0.8, N))
    if N > 3:
        delta[rng.integers(0, N)] = 0.0
    v = rng.normal(0, 25, N)
    t = run_tau(delta, v, dv, 1.2e4, 1.45)
    ref = _mp_tau_lattice(delta, v, dv, 1.2e4, 1.45)
    np.testing.assert_allclose(t, ref, rtol=1e-13, atol=1e-300)


def test_minimal_image_when_line_wider_than_box():
    """b > V/2: the definition keeps one image per source, taken in [-V/2, V/2)."""
    mpmath.mp.dps = 30
    N, dv, T0, gamma = 3, 4.0, 2.0e4, 1.3
    delta = np.array([1.3, 0.7, 2.0])
    v = np.array([5.0, -7.5, 1.0])
    t = run_tau(delta, v, dv, T0, gamma)
    V = N * dv
    for i in range(N):
        acc = mpmath.mpf(0)
        for j in range(N):
            T = mpmath.mpf(T0) * mpmath.mpf(delta[j]) ** (gamma - 1)
            b = mpmath.sqrt(2 * KB * T / MH) / 10 ** 5
            w = delta[j] ** 2 * (T / 10 ** 4) ** mpmath.mpf(-0.7) * dv / (mpmath.sqrt(mpmath.pi) * b)
            d = (i - j) * dv - v[j]
            d = d - V * math.floor((d + V / 2) / V)
            assert -V / 2 <= d < V / 2
            acc += w * mpmath.exp(-(mpmath.mpf(d) / b) ** 2)
        assert t[i] == pytest.approx(float(acc), rel=1e-13)
    mpmath.mp.dps = 15
    assert O.min_image(6.0, 12.0) == -6.0 and O.min_image(-6.0, 12.0) == -6.0


def test_windowed_mode_matches_full_sum():
    w = fields.config1()
    sub = w.subset(range(8))
    full = O.tau(sub.delta, sub.vpec, sub.dv, sub.T0, sub.gamma, offsets=sub.offsets)
    win = O.tau(sub.delta, sub.vpec, sub.dv, sub.T0, sub.gamma, offsets=sub.offsets,
                window_k=8.0)
    np.testing.assert_allclose(win, full, rtol=1e-14, atol=0)


def test_ragged_skewers_are_independent():
    w = fields.ragged_workload("t", 5, 16, 200, 1.0, 4.0, 1e4, 2.5e4, 1.1, 1.6,
                               1.0, 0.8, 6.0, seed=9)
    t = O.tau(w.delta, w.vpec, w.dv, w.T0, w.gamma, offsets=w.offsets)
    for s in range(w.n_skewers):
        a, b = w.offsets[s], w.offsets[s + 1]
        ts = O.tau(w.delta[a:b], w.vpec[a:b], w.dv[s], w.T0[s], w.gamma[s])
        np.testing.assert_array_equal(t[a:b], ts)


def test_domain_errors():
    with pytest.raises(O.OracleError) as e:
        run_tau([1.0, -0.1], [0, 0], 2.0, 1e4, 1.5)
    assert e.value.code == O.ORC_EDOMAIN
    with pytest.raises(O.OracleError):
        run_tau([1.0, np.nan], [0, 0], 2.0, 1e4, 1.5)
    with pytest.raises(O.OracleError):
        run_tau([1.0, 1.0], [0, 0], 0.0, 1e4, 1.5)
    assert np.all(run_tau(np.zeros(8), np.zeros(8), 2.0, 1e4, 1.5) == 0.0)


# -------------------------------------------------------------- mean flux
@pytest.mark.parametrize("tau0,F", [(0.5, 0.8), (3.0, 0.75), (1e-3, 0.5)])
def test_mean_flux_uniform_tau(tau0, F):
    A, _ = O.mean_flux_A(np.full(1000, tau0), F)
    assert A == pytest.approx(-math.log(F) / tau0, rel=1e-14)


@pytest.mark.parametrize("a,F", [(0.3, 0.8), (2.0, 0.6)])
def test_mean_flux_two_level(a, F):
    tau = np.array([a, 2 * a] * 500)
    A, _ = O.mean_flux_A(tau, F)
    x = (math.sqrt(1 + 8 * F) - 1) / 2
    assert A == pytest.approx(-math.log(x) / a, rel=1e-14)


def test_mean_flux_against_brentq():
    from scipy.optimize import brentq
    rng = np.random.default_rng(3)
    tau = np.exp(rng.normal(0, 2.0, 20000))
    tau[:2000] = 0.0
    F = 0.7
    A, _ = O.mean_flux_A(tau, F)
    ref = brentq(lambda a: np.mean(np.exp(-a * tau)) - F, 1e-9, 1e3, xtol=1e-16,
                 rtol=4 * np.finfo(float).eps)
    assert A == pytest.approx(ref, rel=1e-13)
    ts, Fo = O.finalise(tau, A)
    assert Fo.mean() == pytest.approx(F, rel=1e-14)
    np.testing.assert_allclose(ts, A * tau, rtol=0)


def test_paper_printed_mean_flux_and_effective_depth():
    g = json.load(open(os.path.join(GOLDEN, "paper_mean_flux.json")))
    tau = np.full(64, 2.0)
    ts, F, A = O.normalise(tau, g["mean_flux"])
    # tau_eff = -ln <F>, equal to the uniform rescaled depth
    assert round(float(ts[0]), g["printed_decimals_tau_eff"]) == g["tau_eff"]
    assert round(-math.log(F.mean()), g["printed_decimals_tau_eff"]) == g["tau_eff"]


def test_mean_flux_no_root():
    tau = np.array([0.0] * 90 + [1.0] * 10)
    with pytest.raises(O.OracleError) as e:
        O.mean_flux_A(tau, 0.85)  # 90% of pixels are fully transmitting
    assert e.value.code == O.ORC_ENOROOT
    A, _ = O.mean_flux_A(tau, 0.95)
    assert A > 0


# -------------------------------------------------------------- gradients
def _tiny(seed=21, S=3, N=256, dv=2.0):
    # N dv / 2 >= 9 b for every source: the box does not clip the lines
    w = fields.small_workload(n_skewers=S, n_pix=N, seed=seed, dv=dv)
    w.delta[5] = 15.0   # one source above the pivot
    w.delta[7] = 0.0    # one empty source
    w.T0[:] = np.array([1.5e4, 1.1e4, 2.2e4][:S], np.float32)
    w.gamma[:] = np.array([1.5, 1.2, 1.6][:S], np.float32)
    return w


def test_tau_grad_closed_form_sum_of_tau():
    """L = sum_i tau_i with resolved lines (theta = 1):
    dL/dDelta_j = tau_ref (T_j/1e4)^-0.7 Delta_j (2 - 0.7 (gamma-1) [Delta_j <= 10]),
    dL/dv = 0, dL/dT0 = -0.7 sum_j n_j / T0, dL/dgamma = -0.7 sum_j n_j ln D_j,
    with n_j = Delta_j^2 (T_j/1e4)^-0.7."""
    w = _tiny()
    g = np.ones(w.n_pix)
    gd, gv, gT, gg = O.tau_grad(w.delta, w.vpec, w.dv, w.T0, w.gamma, g,
                                offsets=w.offsets)
    for s in range(w.n_skewers):
        sl = slice(w.offsets[s], w.offsets[s + 1])
        d = w.delta[sl].astype(float)
        T0, gm = float(w.T0[s]), float(w.gamma[s])
        D = np.minimum(d, 10.0)
        with np.errstate(divide="ignore", invalid="ignore"):
            T = T0 * D ** (gm - 1)
            n = np.where(d > 0, d ** 2 * (T / 1e4) ** -0.7, 0.0)
            slope = np.where(d <= 10.0, 2 - 0.7 * (gm - 1), 2.0)
            expect = np.where(d > 0, n / np.where(d > 0, d, 1) * slope, 0.0)
            lnD = np.where(d > 0, np.log(np.where(d > 0, D, 1)), 0.0)
        np.testing.assert_allclose(gd[sl], expect, rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(gv[sl], 0.0, atol=1e-9 * np.abs(gd[sl]).max())
        assert gT[s] == pytest.approx(-0.7 * n.sum() / T0, rel=1e-11)
        assert gg[s] == pytest.approx(-0.7 * (n * lnD).sum(), rel=1e-10)


def _loss_full(w, delta, vpec, T0, gamma, F_target, target_F):
    t = O.tau(delta, vpec, w.dv, T0, gamma, offsets=w.offsets)
    _, F, _ = O.normalise(t, target_F)
    return float(((F - F_target) ** 2).sum())


def test_tau_grad_against_finite_differences_through_normalisation():
    """L = sum (F - F_t)^2 with A re-solved at every point: the adjoint (oracle
    tau_grad after normalise_backward with implicit A) against central FD."""
    w = _tiny()
    rng = np.random.default_rng(0)
    d0, v0 = w.delta.astype(float), w.vpec.astype(float)
    T0, gm = w.T0.astype(float), w.gamma.astype(float)
    F_t = np.clip(rng.uniform(0.2, 1.0, w.n_pix), 0, 1)
    t = O.tau(d0, v0, w.dv, T0, gm, offsets=w.offsets)
    ts, F, A = O.normalise(t, w.target_F)
    gF = 2 * (F - F_t)
    g = O.normalise_backward(t, A, grad_F=gF, implicit_A=True)
    gd, gv, gT, gg = O.tau_grad(d0, v0, w.dv, T0, gm, g, offsets=w.offsets)
    L = lambda d, v, a, b: _loss_full(w, d, v, a, b, F_t, w.target_F)
    h = 1e-6
    # random directional derivatives in (Delta, v)
    for k in range(3):
        ud = rng.normal(size=w.n_pix) * (d0 > 0) * (np.abs(d0 - 10) > 1e-3)
        uv = rng.normal(size=w.n_pix)
        fd = (L(d0 + h * ud, v0 + h * uv, T0, gm) -
              L(d0 - h * ud, v0 - h * uv, T0, gm)) / (2 * h)
        an = float(gd @ ud + gv @ uv)
        assert an == pytest.approx(fd, rel=2e-6, abs=1e-9)
    # per-skewer T0 and gamma
    for s in range(w.n_skewers):
        e = np.zeros(w.n_skewers)
        e[s] = 1.0
        hT = 1e-6 * T0[s]
        fdT = (L(d0, v0, T0 + hT * e, gm) - L(d0, v0, T0 - hT * e, gm)) / (2 * hT)
        assert gT[s] == pytest.approx(fdT, rel=1e-5, abs=1e-12)
        hg = 1e-6
        fdg = (L(d0, v0, T0, gm + hg * e) - L(d0, v0, T0, gm - hg * e)) / (2 * hg)
        assert gg[s] == pytest.approx(fdg, rel=1e-5, abs=1e-9)
    # sampled coordinates of Delta and v
    for p in rng.choice(np.flatnonzero((d0 > 0) & (np.abs(d0 - 10) > 1e-2)), 6, replace=False):
        e = np.zeros(w.n_pix)
        e[p] = 1.0
        hd = 1e-6 * d0[p]
        fd = (L(d0 + hd * e, v0, T0, gm) - L(d0 - hd * e, v0, T0, gm)) / (2 * hd)
        assert gd[p] == pytest.approx(fd, rel=1e-5, abs=1e-10)
        hv = 1e-3  # km/s; (hv / b)^2 ~ 1e-8 keeps the O(h^2) error small
        fdv = (L(d0, v0 + hv * e, T0, gm) - L(d0, v0 - hv * e, T0, gm)) / (2 * hv)
        assert gv[p] == pytest.approx(fdv, rel=1e-5, abs=1e-7 * np.abs(gv).max())


def test_implicit_A_makes_T0_gradient_vanish_for_mean_flux_loss():
    """With A re-solved, tau' depends on T0 only through a uniform factor when
    T0 is common to all skewers... of sum F, which is pinned to P Fbar: d(sum F)/dT0 = 0."""
    w = _tiny(S=1)
    t = O.tau(w.delta, w.vpec, w.dv, w.T0, w.gamma, offsets=w.offsets)
    _, F, A = O.normalise(t, w.target_F)
    g = O.normalise_backward(t, A, grad_F=np.ones(w.n_pix), implicit_A=True)
    gd, gv, gT, gg = O.tau_grad(w.delta, w.vpec, w.dv, w.T0, w.gamma, g,
                                offsets=w.offsets)
    assert abs(gT[0]) < 1e-12 and np.abs(gd).max() < 1e-12


def test_normalise_backward_against_fd():
    rng = np.random.default_rng(4)
    tau = np.exp(rng.normal(0, 1.5, 200))
    tau[:5] = 0.0
    cF = rng.normal(size=200)
    cT = rng.normal(size=200)
    F_bar = 0.7

    def L(t):
        ts, F, _ = O.normalise(t, F_bar)
        return float(cF @ F + cT @ ts)

    ts, F, A = O.normalise(tau, F_bar)
    g = O.normalise_backward(tau, A, grad_F=cF, grad_tau_scaled=cT, implicit_A=True)
    h = 1e-6
    for p in [6, 7, 50, 199]:  # tau > 0 (a zero pixel cannot go negative)
        e = np.zeros(200)
        e[p] = 1.0
        hp = h * max(tau[p], 1.0)
        fd = (L(tau + hp * e) - L(tau - hp * e)) / (2 * hp)
        assert g[p] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    # frozen A: just A * G
    g0 = O.normalise_backward(tau, A, grad_F=cF, grad_tau_scaled=cT, implicit_A=False)
    np.testing.assert_allclose(g0, A * (cT - F * cF), rtol=1e-14)


def test_tau_at_chosen_pixels_is_the_full_sum():
    """tau_at evaluates the same full sum as tau for chosen pixels of one
    skewer (same terms, same order): bitwise equal, including the first and
    last pixels where the minimal image wraps, on a ragged batch."""
    w = fields.ragged_workload("mix", 5, 40, 700, 1.0, 4.0, 1e4, 2.5e4, 1.1, 1.6, 1.0, 0.8, 6.0,
                               seed=61)
    full = O.tau(w.delta, w.vpec, w.dv, w.T0, w.gamma, offsets=w.offsets, tau_ref=w.tau_ref,
                 delta_pivot=w.delta_pivot)
    for s in range(w.n_skewers):
        a, b = int(w.offsets[s]), int(w.offsets[s + 1])
        pick = np.unique(np.r_[0, 1, b - a - 2, b - a - 1,
                               np.random.default_rng(s).integers(0, b - a, 7)])
        got = O.tau_at(w.delta, w.vpec, w.dv, w.T0, w.gamma, w.offsets, s, pick,
                       tau_ref=w.tau_ref, delta_pivot=w.delta_pivot)
        assert np.array_equal(got, full[a + pick])
    with pytest.raises(O.OracleError):
        O.tau_at(w.delta, w.vpec, w.dv, w.T0, w.gamma, w.offsets, 0, [int(np.diff(w.offsets)[0])])
