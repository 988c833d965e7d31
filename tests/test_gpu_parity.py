"""GPU parity of the optical-depth path against the FP64 CPU oracle.

Every case runs the HIP library through its C ABI and compares element by
element with the oracle on the same seeded inputs, at the tolerances stated in
gpu_util.py.  Full-size workloads (4096 x 4096, 20,000 ragged skewers, the
512 x 512 x 4096 box) run in the launch configuration the benchmark times and
are compared on sampled skewers that the oracle computes in full.  The
mean-flux constant is checked two ways: the condition it solves,
g(A) = <exp(-A tau)> - target = 0, evaluated in FP64 on the GPU's own raw tau
over every pixel (a property, no oracle value; |g| <= 1e-7 A |g'|), and the
oracle's own chain over the whole batch (its windowed k = 8 tau, its own A at
1e-7, and the globally normalised F on the sampled skewers at 1e-6).  F is
also compared on a subset that each side normalises on its own.  No oracle
input comes from the GPU.
"""
import math

import numpy as np
import pytest

from gpu_util import (OnDevice, assert_F_close, assert_mean_flux_root,
                      assert_subset_flux, assert_tau_close, gpu_normalise, gpu_tau,
                      mean_flux_residual_chunked, to_dev, A_REL)
from oracle import oracle as O
from synth import fields

pytestmark = pytest.mark.gpu


def oracle_tau(w, window_k=0.0):
    return O.tau(w.delta, w.vpec, w.dv, w.T0, w.gamma, offsets=w.offsets,
                 tau_ref=w.tau_ref, delta_pivot=w.delta_pivot, window_k=window_k)


def flags():
    from paper_1105_4747_amd import lyaf as L
    return L


@pytest.fixture(scope="module")
def c1():
    return fields.config1()


# ---------------------------------------------------------------- tau
@pytest.mark.parametrize("mode", ["window", "plain", "per_skewer", "full_k0"])
def test_tau_config1_all_forms(c1, mode):
    L = flags()
    fl = {"window": 0, "plain": L.FLAG_PLAIN,
          "per_skewer": L.FLAG_PER_SKEWER, "full_k0": 0}[mode]
    k = 0.0 if mode == "full_k0" else None
    print(f"case: C1 64x1024 mode={mode}", flush=True)
    got = gpu_tau(c1, flags=fl, window_k=k).cpu().numpy()
    ref = oracle_tau(c1)
    worst = assert_tau_close(got, ref, f"C1 {mode}")
    print(f"C1 {mode}: worst err/tol {worst:.3f}")


@pytest.mark.parametrize("n_skewers,n_pix,dv", [(8, 256, 2.0), (3, 100, 3.0), (5, 17, 1.0),
                                                (4, 1, 2.0), (2, 600, 1.0), (6, 2000, 4.0)])
def test_tau_small_and_ragged_tails(n_skewers, n_pix, dv):
    w = fields.small_workload(n_skewers=n_skewers, n_pix=n_pix, seed=n_pix, dv=dv)
    print(f"case: {w.name} dv={dv}", flush=True)
    got = gpu_tau(w).cpu().numpy()
    assert_tau_close(got, oracle_tau(w), w.name)


def test_tau_ragged_batch_with_empty_skewers():
    base = fields.ragged_workload("rag", 9, 1, 3000, 1.0, 4.0, 1e4, 2.5e4, 1.1, 1.6, 1.0,
                                  0.8, 6.0, seed=17)
    lengths = np.diff(base.offsets).copy()
    lengths[[0, 4]] = 0          # empty skewers inside the batch
    lengths[2] = 1
    lengths[6] = 257             # one past a tile
    off = np.zeros(len(lengths) + 1, np.int64)
    off[1:] = np.cumsum(lengths)
    rng = np.random.default_rng(5)
    P = int(off[-1])
    D, v = fields.lognormal_skewers(lengths, 1.0, seed=23)
    D[rng.integers(0, P, 40)] = 0.0       # empty pixels
    D[rng.integers(0, P, 10)] *= 50.0     # far above the pivot
    w = fields.Workload("ragged-edge", D, v, off, base.dv, base.T0, base.gamma, 0.8, 6.0)
    print(f"case: ragged edge lengths={lengths.tolist()}", flush=True)
    got = gpu_tau(w).cpu().numpy()
    assert_tau_close(got, oracle_tau(w), "ragged-edge")


def test_tau_cold_unresolved_sources_and_inverted_relation():
    """Unresolved lines (b well below dv), gamma < 1, pivot disabled, and an
    all-empty skewer."""
    w = fields.small_workload(n_skewers=6, n_pix=1500, seed=31, dv=4.0, sigma_lnD=2.5)
    w.gamma[:] = np.array([1.6, 1.6, 0.7, 1.3, 1.6, 1.6], np.float32)
    w.T0[:] = np.array([3e3, 1e4, 1e4, 2e4, 500.0, 1e4], np.float32)
    w.delta[5 * 1500:] = 0.0
    for pivot in (10.0, math.inf):
        w.delta_pivot = pivot
        print(f"case: cold sources pivot={pivot}", flush=True)
        got = gpu_tau(w).cpu().numpy()
        ref = oracle_tau(w)
        assert np.all(got[5 * 1500:] == 0.0)
        assert_tau_close(got, ref, f"cold pivot={pivot}")


@pytest.mark.parametrize("shape", [0, 4, 5])
def test_tau_recurrence_shape_near_and_past_its_limit(shape):
    """The recurrence shapes (4: 4 targets per lane, limit a <= 1; 5: 8 targets,
    limit a <= 0.45) on isothermal skewers whose lines are narrow against the
    pixels: a = dv sqrt(log2 e) / b of 0.37, 0.43 (shape 5 close to its limit),
    0.93 (shape 4 close to its limit, shape 5 past it) and 1.08 (both fall back
    to the direct form), against the oracle; shape 0 on the same skewers for
    comparison."""
    from paper_1105_4747_amd import lyaf as L
    w = fields.small_workload(n_skewers=4, n_pix=5000, seed=41, dv=4.0, sigma_lnD=1.5)
    w.gamma[:] = 1.0
    w.T0[:] = np.array([1e4, 7.6e3, 1.6e3, 1.2e3], np.float32)
    print(f"case: narrow lines shape={shape}", flush=True)
    got = gpu_tau(w, flags=L.FLAG_SHAPE(shape)).cpu().numpy()
    assert_tau_close(got, oracle_tau(w), f"narrow lines shape {shape}")


def test_tau_is_linear_in_tau_ref_and_deterministic(c1):
    a = gpu_tau(c1).cpu().numpy()
    b = gpu_tau(c1).cpu().numpy()
    assert np.array_equal(a, b), "two runs differ bitwise"
    c = gpu_tau(c1, tau_ref=2.0).cpu().numpy()
    np.testing.assert_allclose(c, 2 * a, rtol=3e-7)


# ---------------------------------------------------------------- mean flux
def test_normalise_config1(c1):
    d = OnDevice(c1)
    raw = gpu_tau(c1, d=d)
    ts, F, A = gpu_normalise(raw, c1.target_F)
    raw_np = raw.cpu().numpy().astype(np.float64)
    # (i) root-find parity on the same input: the oracle's raw tau, rounded to
    # float32, normalised by both sides
    ref = oracle_tau(c1)
    ref32 = ref.astype(np.float32)
    _, _, A32 = gpu_normalise(to_dev(ref32), c1.target_F)
    A_same, _ = O.mean_flux_A(ref32.astype(np.float64), c1.target_F)
    assert abs(float(A32.cpu()) / A_same - 1) <= A_REL
    assert_mean_flux_root(raw_np, float(A.cpu()), c1.target_F, "C1 A on its own tau")
    # (ii) end-to-end against the oracle's own tau
    ts_ref, F_ref, A_ref = O.normalise(ref, c1.target_F)
    assert_tau_close(ts.cpu().numpy(), ts_ref, "C1 tau'")
    e = assert_F_close(F.cpu().numpy(), F_ref, "C1 F")
    assert abs(float(F.double().mean().cpu()) - c1.target_F) < 1e-6
    print(f"C1 normalise: A={float(A.cpu()):.12g} ref={A_ref:.12g} max|dF|={e:.2e}")
    from paper_1105_4747_amd import lyaf as L
    assert L.status_read() == 0


@pytest.mark.parametrize("tau0,F", [(0.7, 0.8), (5.0, 0.3)])
def test_normalise_uniform_closed_form(tau0, F):
    import torch
    raw = torch.full((100003,), tau0, device="cuda:0", dtype=torch.float32)
    ts, Fo, A = gpu_normalise(raw, F)
    assert abs(float(A.cpu()) / (-math.log(F) / float(np.float32(tau0))) - 1) <= 1e-12
    assert abs(float(Fo[0].cpu()) - F) <= 1e-7


def test_normalise_status_no_root_and_domain():
    import torch
    from paper_1105_4747_amd import lyaf as L
    L.status_read()
    raw = torch.zeros(1000, device="cuda:0")
    raw[:50] = 1.0                     # 95% of pixels fully transmitting
    gpu_normalise(raw, 0.8)
    assert L.status_read() & L.STATUS_NOROOT
    raw[0] = -1.0
    gpu_normalise(raw, 0.8)
    assert L.status_read() & L.STATUS_DOMAIN
    assert L.status_read() == 0        # read clears


SAMPLE_N = 8192  # pixels the root-find's first stage sees: floor(k P / N), k < N


def _sample_blind(rng, P):
    """tau over P = 4 N pixels with every sampled pixel (k P / N = 4k) zero."""
    import torch
    raw = (np.exp(rng.normal(0.0, 1.0, P)) * 0.4).astype(np.float32)
    raw[::4] = 0.0
    return raw, torch.from_numpy(raw).to("cuda:0")


def test_normalise_sample_sees_only_zeros():
    """The first stage converges on evenly spaced pixels; here all of them are
    zero and the signal lies between them.  The passes over every pixel must
    still reach the root, or say that they did not (NOCONV): never a wrong A
    with a clean status."""
    from paper_1105_4747_amd import lyaf as L
    rng = np.random.default_rng(7)
    raw, d = _sample_blind(rng, 4 * SAMPLE_N)
    L.status_read()
    ts, F, A = gpu_normalise(d, 0.8)
    st = L.status_read()
    A_ref, _ = O.mean_flux_A(raw.astype(np.float64), 0.8)
    print(f"blind sample: A={float(A.cpu()):.12g} ref={A_ref:.12g} status={st}")
    if st == 0:
        assert abs(float(A.cpu()) / A_ref - 1) <= A_REL
    else:
        assert st == L.STATUS_NOCONV


@pytest.mark.parametrize("other", [1.08, 1.2, 1.6])
def test_normalise_from_a_biased_sample(other):
    """Every sampled pixel (4k of P = 4 N) has tau = 1 and the others ``other``:
    the sample's root settles away from the batch's by ~6 %, ~15 % and ~40 %.
    The first full pass's series step is then taken (~6 %) or, past a tenth of
    A, refused for Halley steps until a later series step is accepted; A must
    reach the oracle's root with a clean status either way."""
    import torch
    from paper_1105_4747_amd import lyaf as L
    P = 4 * SAMPLE_N
    raw = np.full(P, other, np.float32)
    raw[::4] = 1.0
    L.status_read()
    ts, F, A = gpu_normalise(torch.from_numpy(raw).to("cuda:0"), 0.8)
    st = L.status_read()
    A_ref, _ = O.mean_flux_A(raw.astype(np.float64), 0.8)
    print(f"biased sample ({other}): A={float(A.cpu()):.15g} ref={A_ref:.15g} status={st}")
    assert st == 0
    assert abs(float(A.cpu()) / A_ref - 1) <= A_REL
    assert np.allclose(ts.cpu().numpy(), float(A.cpu()) * raw, rtol=1e-7, atol=0)


def test_normalise_root_and_domain_checks_cover_unsampled_pixels():
    """No root, or an invalid value, that only the pixels outside the sample
    reveal: the full passes report it."""
    import torch
    from paper_1105_4747_amd import lyaf as L
    P = 4 * SAMPLE_N
    L.status_read()
    raw = torch.zeros(P, device="cuda:0")
    raw[::4] = 1.0                      # the sample alone has a root for F = 0.7
    gpu_normalise(raw, 0.7)             # 75% of all pixels transmit fully: none
    assert L.status_read() == L.STATUS_NOROOT
    rng = np.random.default_rng(8)
    good = torch.from_numpy((np.exp(rng.normal(0.0, 1.0, P)) * 0.4).astype(np.float32))
    good = good.to("cuda:0")
    gpu_normalise(good, 0.7)
    assert L.status_read() == 0
    good[4 * 1000 + 1] = float("nan")   # not a sampled pixel
    gpu_normalise(good, 0.7)
    assert L.status_read() & L.STATUS_DOMAIN


def test_tau_status_domain():
    from paper_1105_4747_amd import lyaf as L
    w = fields.small_workload(n_skewers=2, n_pix=64, seed=2)
    L.status_read()
    w.delta[3] = -0.5
    gpu_tau(w)
    assert L.status_read() & L.STATUS_DOMAIN
    w.delta[3] = 1.0
    w.dv[1] = 0.0
    gpu_tau(w)
    assert L.status_read() & L.STATUS_DOMAIN


# ---------------------------------------------------------------- full sizes
def _whole_batch_chain(w, F_gpu, A_gpu, sel, what):
    """The oracle's own chain over the whole batch: windowed (k = 8) FP64 tau,
    its root A and F = exp(-A tau).  The GPU's globally normalised F must match
    on the sampled pixels ``sel``, and A_gpu the oracle's A."""
    import time
    t0 = time.perf_counter()
    raw_ref = oracle_tau(w, window_k=8.0)
    print(f"{what}: oracle windowed tau over {w.n_pix} px in {time.perf_counter() - t0:.1f} s",
          flush=True)
    A_ref, _ = O.mean_flux_A(raw_ref, w.target_F)
    F_ref = np.exp(-A_ref * raw_ref[sel])
    del raw_ref
    eF = assert_F_close(F_gpu[sel], F_ref, f"{what} globally normalised F")
    relA = abs(A_gpu / A_ref - 1.0)
    print(f"{what}: |A_gpu / A_oracle - 1| = {relA:.2e}, max|dF| = {eF:.2e}", flush=True)
    assert relA <= A_REL, f"{what}: A_gpu {A_gpu:.15g} vs oracle chain {A_ref:.15g}"
    return relA, eF


@pytest.mark.slow
def test_config2_full_size_sampled():
    """4096 x 4096 in the benchmark's launch shape; skewers 0..63 plus 32 drawn
    at random are compared in full.  A as the root of the mean-flux condition
    on the GPU's 16.8M raw tau values, and against the oracle's own chain over
    the whole batch, whose F the GPU's globally normalised F matches on the
    sampled skewers."""
    w = fields.config2()
    print(f"case: {w.name}", flush=True)
    d = OnDevice(w)
    raw = gpu_tau(w, d=d)
    ts, F, A = gpu_normalise(raw, w.target_F)
    raw_np = raw.cpu().numpy()
    F_np = F.cpu().numpy()
    A_gpu = float(A.cpu())
    rng = np.random.default_rng(2)
    pick = np.concatenate([np.arange(64), rng.choice(np.arange(64, 4096), 32, replace=False)])
    sub = w.subset(pick)
    ref = oracle_tau(sub)
    sel = np.concatenate([np.arange(w.offsets[s], w.offsets[s + 1]) for s in pick])
    worst = assert_tau_close(raw_np[sel], ref, "C2 sampled raw tau")
    rA = assert_mean_flux_root(raw_np, A_gpu, w.target_F, "C2 A")
    eF = assert_subset_flux(raw_np[sel], ref, w.target_F, "C2 sampled F")
    _whole_batch_chain(w, F_np, A_gpu, sel, "C2")
    print(f"C2: worst tau err/tol {worst:.3f}, root residual {rA:.2e} of A, "
          f"subset max|dF| {eF:.2e}")


@pytest.mark.slow
def test_config3_ragged_full_size_sampled():
    w = fields.config3()
    print(f"case: {w.name} P={w.n_pix}", flush=True)
    raw = gpu_tau(w)
    ts, F, A = gpu_normalise(raw, w.target_F)
    raw_np = raw.cpu().numpy()
    F_np = F.cpu().numpy()
    A_gpu = float(A.cpu())
    lens = np.diff(w.offsets)
    rng = np.random.default_rng(3)
    pick = np.unique(np.concatenate([[int(np.argmin(lens)), int(np.argmax(lens))],
                                     np.argsort(w.dv)[:3], np.argsort(w.dv)[-3:],
                                     rng.choice(w.n_skewers, 18, replace=False)]))
    sub = w.subset(pick)
    ref = oracle_tau(sub)
    sel = np.concatenate([np.arange(w.offsets[s], w.offsets[s + 1]) for s in pick])
    worst = assert_tau_close(raw_np[sel], ref, "C3 sampled raw tau")
    rA = assert_mean_flux_root(raw_np, A_gpu, w.target_F, "C3 A")
    assert_subset_flux(raw_np[sel], ref, w.target_F, "C3 sampled F")
    _whole_batch_chain(w, F_np, A_gpu, sel, "C3")
    print(f"C3: worst tau err/tol {worst:.3f}, root residual {rA:.2e} of A")


@pytest.mark.slow
def test_config4_box_sampled():
    """512 x 512 skewers of 4096 px from one 3D lognormal field (generated on
    the GPU), the global mean-flux rescale, 48 sampled skewers in full."""
    import torch
    w = fields.config4(device="cuda:0")
    print(f"case: {w.name} P={w.n_pix}", flush=True)
    d = OnDevice(w)
    raw = gpu_tau(w, d=d)
    ts, F, A = gpu_normalise(raw, w.target_F)
    rng = np.random.default_rng(4)
    pick = np.sort(rng.choice(w.n_skewers, 48, replace=False))
    sel = np.concatenate([np.arange(w.offsets[s], w.offsets[s + 1]) for s in pick])
    sel_t = torch.from_numpy(sel).to("cuda:0")
    sub = fields.Workload("C4 sample", w.delta[sel_t].cpu().numpy(), w.vpec[sel_t].cpu().numpy(),
                          np.arange(len(pick) + 1, dtype=np.int64) * 4096, w.dv[pick],
                          w.T0[pick], w.gamma[pick], w.target_F, w.window_k)
    ref = oracle_tau(sub)
    worst = assert_tau_close(raw[sel_t].cpu().numpy(), ref, "C4 sampled raw tau")
    # A at the A bar: the condition it solves, g(A) = <exp(-A tau)> - target = 0,
    # evaluated in FP64 over all 1.07e9 raw values (|g| <= 1e-7 A |g'(A)|)
    A_gpu = float(A.cpu())
    g, dg = mean_flux_residual_chunked(raw, A_gpu, w.target_F)
    rA = abs(g) / (A_gpu * dg)
    assert rA <= A_REL, f"C4 A: g(A) = {g:.3g}, allowed {A_REL * A_gpu * dg:.3g}"
    eF = assert_subset_flux(raw[sel_t].cpu().numpy(), ref, w.target_F, "C4 sampled F")
    print(f"C4: worst tau err/tol {worst:.3f}, root residual {rA:.2e} of A, "
          f"max|dF| {eF:.2e}")
    del d, raw, ts, F, A


@pytest.mark.slow
def test_tau_at_the_maximum_skewer_length():
    """One skewer of 2^24 pixels, the longest the library accepts (pixel
    offsets are formed exactly in FP32): 160 pixels, both ends (where the
    minimal image wraps) and 128 drawn at random, against the oracle's full sum
    at those pixels, and A as the root of the mean-flux condition on the GPU's
    16.8M raw tau values."""
    n = 1 << 24
    w = fields.uniform_workload("1 x 2^24", 1, n, 2.0, 1.2, 2.0e4, 1.3, 0.75, 6.0, seed=9)
    print(f"case: {w.name}", flush=True)
    raw = gpu_tau(w)
    ts, F, A = gpu_normalise(raw, w.target_F)
    raw_np = raw.cpu().numpy()
    pick = np.unique(np.r_[np.arange(16), np.arange(n - 16, n),
                           np.random.default_rng(9).integers(0, n, 128)])
    ref = O.tau_at(w.delta, w.vpec, w.dv, w.T0, w.gamma, w.offsets, 0, pick,
                   tau_ref=w.tau_ref, delta_pivot=w.delta_pivot)
    worst = assert_tau_close(raw_np[pick], ref, "2^24 sampled raw tau")
    rA = assert_mean_flux_root(raw_np, float(A.cpu()), w.target_F, "2^24 A")
    print(f"2^24: worst tau err/tol {worst:.3f}, root residual {rA:.2e} of A")
