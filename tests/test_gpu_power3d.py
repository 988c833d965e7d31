"""GPU parity of the 3D flux power spectrum reconstruction of eq. (7)
(lyaf_flux_power_3d) against the FP64 oracle (oracle/flux_power_3d.py),
through the C ABI.

The library computes in FP64 throughout; the shell sums are FP64 atomics in
LDS, so they agree with the oracle to rounding.  Bar, per shell: counts exact;
mean |k| within 1e-12 relative; mean P_box within 1e-10 relative; mean P_true
within 1e-10 of that shell's mean P_box (P_true is a difference of two terms
of P_box's size, so its error scales with P_box).  At the full size, where the
oracle's full grid is too large, properties that hold at any size: the shell
counts against a brute-force count of the half-spectrum's modes, Parseval's
identity for the total box power, and the total of P_true, which eq. (7) fixes
at -L^2 S P_N / n for unit weights on distinct columns."""
import math

import numpy as np
import pytest

from oracle import flux_power_3d as P3

pytestmark = pytest.mark.gpu

KMEAN_REL, PBOX_REL, PTRUE_REL = 1e-12, 1e-10, 1e-10


def _run(F, mean_F, sx, sy, n, L, n_bins, weights=None, p_noise=0.0):
    import torch
    from paper_1105_4747_amd import lyaf as Lb
    dev = torch.device("cuda:0")
    Fd = torch.from_numpy(np.ascontiguousarray(F, dtype=np.float32).reshape(-1)).to(dev)
    wd = None if weights is None else torch.from_numpy(
        np.ascontiguousarray(weights, dtype=np.float64)).to(dev)
    out = [torch.full((n_bins,), float("nan"), device=dev, dtype=torch.float64)
           for _ in range(4)]
    Lb.flux_power_3d(Fd, mean_F, sx, sy, n, L, n_bins, *out, weights=wd, p_noise=p_noise)
    torch.cuda.synchronize()
    assert Lb.status_read() == 0
    return [o.cpu().numpy() for o in out]


def _flux(S, n, seed):
    rng = np.random.default_rng(seed)
    return np.exp(-np.exp(rng.normal(-1.0, 1.0, (S, n)))).astype(np.float32)


def _compare(got, ref):
    cnt, km, pt, pb = got
    rc, rk, rpt, rpb = ref
    assert np.array_equal(cnt, rc), "shell counts differ"
    scale_b = np.abs(rpb)
    ek = np.max(np.abs(km - rk) / np.maximum(np.abs(rk), 1e-300))
    eb = np.max(np.abs(pb - rpb) / np.maximum(scale_b, 1e-300))
    et = np.max(np.abs(pt - rpt) / np.maximum(scale_b, 1e-300))
    print(f"  k_mean rel {ek:.1e}, P_box rel {eb:.1e}, P_true / P_box {et:.1e}", flush=True)
    assert ek <= KMEAN_REL and eb <= PBOX_REL and et <= PTRUE_REL


def _check(n, S, seed, L=100.0, weights=False, p_noise=0.0, n_bins=None, cols=None):
    rng = np.random.default_rng(seed)
    sx, sy = cols if cols is not None else (rng.integers(0, n, S), rng.integers(0, n, S))
    F = _flux(len(sx), n, seed)
    w = rng.uniform(0.5, 2.0, len(sx)) if weights else None
    nb = n_bins or int(math.floor(math.sqrt(3) * n / 2)) + 3
    print(f"power3d: n={n} S={len(sx)} seed={seed} weights={weights} P_N={p_noise} "
          f"bins={nb}", flush=True)
    got = _run(F, 0.7, sx, sy, n, L, nb, w, p_noise)
    ref = P3.flux_power_3d(F.astype(np.float64), 0.7, sx, sy, n, L, nb, w, p_noise)
    _compare(got, ref)
    return got


@pytest.mark.parametrize("n", [4, 8, 16, 32, 64, 128])
def test_random_sight_lines_every_size(n):
    """Random columns with repeats (two sight-lines in one column add up) on
    every grid size up to 128."""
    _check(n, 3 * n, seed=n)


def test_weights_noise_and_few_bins():
    """Per-sight-line weights, a noise power, and fewer shells than the grid
    has (modes past the last shell are dropped)."""
    _check(32, 70, seed=3, weights=True, p_noise=0.37)
    _check(32, 70, seed=4, n_bins=9)


def test_crowded_rows_and_one_sight_line():
    """A row holding 20 sight-lines (more than the kernel keeps in registers)
    and a single sight-line (P_true = -P_N L^2 / n^4 on every mode)."""
    n = 64
    sx = np.concatenate([np.arange(20) * 3, [5, 40]])
    sy = np.concatenate([np.full(20, 7), [1, 63]])
    _check(n, 0, seed=6, cols=(sx, sy), p_noise=0.2)
    cnt, km, pt, pb = _check(n, 0, seed=7, cols=(np.array([9]), np.array([33])), p_noise=0.5)
    L = 100.0
    live = cnt > 0
    assert np.allclose(pt[live], -0.5 * L ** 2 / n ** 4, rtol=1e-12, atol=0)


def test_identical_sight_lines_cancel():
    """Every sight-line carrying the same spectrum: the box power is exactly the
    aliasing term, so P_true = 0 up to rounding (the oracle's pin, on the GPU)."""
    n, S = 32, 25
    rng = np.random.default_rng(2)
    cols = rng.choice(n * n, S, replace=False)
    sx, sy = cols // n, cols % n
    F = np.tile(_flux(1, n, 5), (S, 1))
    nb = int(math.floor(math.sqrt(3) * n / 2)) + 1
    cnt, km, pt, pb = _run(F, 0.7, sx, sy, n, 100.0, nb)
    assert np.max(np.abs(pt)) <= 1e-12 * np.max(np.abs(pb))


def test_full_size_workload_properties():
    """The benchmark's workload (1024 pixels per side, 6,250 sight-lines on
    distinct columns, synthetic flux): shell counts against a brute-force count
    of the half-spectrum's modes, Parseval for the total box power and the
    total of P_true, in FP64 on the host."""
    from synth import fields
    w = fields.power3d_workload()
    n, L, S = w.n, w.box, len(w.sx)
    nb = int(math.floor(math.sqrt(3) * n / 2)) + 1
    print(f"power3d: {w.name}", flush=True)
    cnt, km, pt, pb = _run(w.F, w.mean_F, w.sx, w.sy, n, L, nb, p_noise=w.p_noise)
    # brute-force shell counts, one mx plane at a time
    m = np.fft.fftfreq(n, d=1.0 / n)
    mz = np.arange(n // 2 + 1, dtype=np.float64)
    c = np.where((mz == 0) | (mz == n // 2), 1.0, 2.0)
    ref_cnt = np.zeros(nb)
    for a in m:
        b = np.floor(np.sqrt(a * a + m[:, None] ** 2 + mz[None, :] ** 2)).astype(np.int64)
        ref_cnt += np.bincount(b.ravel(), weights=np.broadcast_to(c, b.shape).ravel(),
                               minlength=nb)[:nb]
    assert np.array_equal(cnt, ref_cnt)
    assert cnt.sum() == n ** 3
    delta = w.F.astype(np.float64).reshape(S, n) / w.mean_F - 1.0
    sum_d2 = float(np.sum(delta * delta))
    tot_box = float(np.sum(cnt * pb))
    want_box = L ** 3 / n ** 3 * sum_d2
    tot_true = float(np.sum(cnt * pt))
    want_true = -L ** 2 * S * w.p_noise / n
    print(f"  total P_box {tot_box:.6e} vs {want_box:.6e}; total P_true {tot_true:.6e} "
          f"vs {want_true:.6e}", flush=True)
    assert abs(tot_box / want_box - 1) <= 1e-11
    assert abs(tot_true - want_true) <= 1e-10 * tot_box
