"""GPU parity of the skewer-only field synthesis (lyaf_field_skewers) against
the FP64 oracle (oracle/field_synthesis.py), through the C ABI.

Bar (per field, over the compared sight-lines): max |f_gpu - f_ref| <=
FIELD_TOL * rms(f_ref).  The my transform runs in FP32 (relative rms error
~u log2 n per value, u = 2^-24, plus the rounding of the FP32 multipliers and
of the stored intermediate); the mx sums and the z transform run in FP64 and
only add and rotate those errors, so each output carries an error of a few
u times the field's rms, and the largest of ~10^6 values a few times that.
FIELD_TOL = 1e-5 leaves a factor of ~5 over the worst measured case."""
import math

import numpy as np
import pytest

from oracle import field_synthesis as FS

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-5


def _modes(N, seed):
    rng = np.random.default_rng(seed)
    shape = (N, N, N // 2 + 1)
    return (rng.normal(size=shape) + 1j * rng.normal(size=shape)).astype(np.complex64)


def _table(N, L, n=200, seed=3, full=True):
    """A positive table reaching past the grid's largest |k| (or stopping short
    of it when full=False, so that high-k modes are dropped)."""
    kmax = math.sqrt(3) * math.pi * N / L
    dk = (1.02 if full else 0.5) * kmax / (n - 1)
    rng = np.random.default_rng(seed)
    k = np.arange(n) * dk
    return (1.0 + k) ** -1.5 * (1.0 + 0.2 * rng.random(n)), dk


def _run(modes, pk, dk, amp, L, kF, Ep, sx, sy):
    import torch
    from paper_1105_4747_amd import lyaf as Lb
    dev = torch.device("cuda:0")
    N = modes.shape[0]
    m = torch.from_numpy(np.ascontiguousarray(modes)).to(dev) if isinstance(modes, np.ndarray) \
        else modes
    p = torch.from_numpy(np.ascontiguousarray(pk, dtype=np.float64)).to(dev)
    S = len(sx)
    b = torch.full((S, N), float("nan"), device=dev, dtype=torch.float32)
    v = torch.full((S, N), float("nan"), device=dev, dtype=torch.float32)
    Lb.field_skewers(m, p, sx, sy, b, v, N, L, amp, kF, Ep, dk)
    torch.cuda.synchronize()
    assert Lb.status_read() == 0
    return b.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)


def _assert_close(name, got, ref):
    scale = float(np.sqrt(np.mean(ref * ref)))
    err = float(np.max(np.abs(got - ref))) / max(scale, 1e-300)
    print(f"  {name}: max err / rms = {err:.2e} (bar {FIELD_TOL:.0e})", flush=True)
    assert np.all(np.isfinite(got))
    assert err <= FIELD_TOL


def _check(N, sx, sy, seed=1, L=50.0, kF=3.0, Ep=80.0, amp=2.0, full=True):
    print(f"field synthesis: N={N} S={len(sx)} kF={kF} seed={seed}", flush=True)
    modes = _modes(N, seed)
    pk, dk = _table(N, L, full=full)
    b, v = _run(modes, pk, dk, amp, L, kF, Ep, sx, sy)
    rb, rv = FS.skewer_fields(modes.astype(np.complex128), pk, dk, amp, L, kF, Ep, sx, sy)
    _assert_close("delta_b", b, rb)
    _assert_close("v_z", v, rv)
    return b, v


@pytest.mark.parametrize("N", [4, 8, 16, 32, 64, 128])
def test_every_column_of_small_grids(N):
    """Every column of the grid (every row in use, every group full)."""
    sx, sy = np.repeat(np.arange(N), N), np.tile(np.arange(N), N)
    _check(N, sx, sy, seed=N)


def test_random_columns_with_repeats_and_crowded_rows():
    """Random columns, repeated columns (identical outputs), and one row with 21
    sight-lines (three groups of the mx sum)."""
    N = 64
    rng = np.random.default_rng(5)
    sx = np.concatenate([rng.integers(0, N, 150), np.arange(21) * 3, [7, 7]]).astype(np.int32)
    sy = np.concatenate([rng.integers(0, N, 150), np.full(21, 9), [11, 11]]).astype(np.int32)
    b, v = _check(N, sx, sy, seed=9)
    assert np.array_equal(b[-1], b[-2]) and np.array_equal(v[-1], v[-2])


def test_no_filter_short_table_and_one_sight_line():
    """k_F = +inf (no smoothing), a table that ends inside the grid's k range
    (modes past it dropped), and a single sight-line."""
    N = 32
    _check(N, np.array([5]), np.array([30]), seed=3, kF=math.inf)
    rng = np.random.default_rng(2)
    _check(N, rng.integers(0, N, 40), rng.integers(0, N, 40), seed=4, full=False)


def test_one_entry_table_keeps_only_the_mean_mode():
    """A table of one entry gives power only at k = 0: delta_b is the constant
    amp sqrt(P0) Re g(0) / N^3 and the velocity is zero (eq. 3 has no k = 0 term)."""
    N = 16
    modes = _modes(N, 6)
    sx, sy = np.array([0, 3, 15]), np.array([2, 2, 9])
    b, v = _run(modes, np.array([4.0]), 0.1, 1.5, 10.0, 2.0, 50.0, sx, sy)
    want = 1.5 * 2.0 * float(modes[0, 0, 0].real) / N ** 3
    assert np.allclose(b, want, rtol=1e-6, atol=0)
    assert np.all(v == 0.0)


def test_sight_line_order_does_not_matter():
    """Outputs follow the caller's order of sight-lines (a permutation of the
    columns permutes the rows of the output exactly)."""
    N = 32
    rng = np.random.default_rng(8)
    sx, sy = rng.integers(0, N, 60), rng.integers(0, N, 60)
    modes = _modes(N, 2)
    pk, dk = _table(N, 30.0)
    b1, v1 = _run(modes, pk, dk, 1.0, 30.0, 2.5, 40.0, sx, sy)
    perm = rng.permutation(60)
    b2, v2 = _run(modes, pk, dk, 1.0, 30.0, 2.5, 40.0, sx[perm], sy[perm])
    assert np.array_equal(b1[perm], b2) and np.array_equal(v1[perm], v2)


def test_full_size_workload_sampled():
    """The benchmark's workload (1024^3 grid, 6,250 sight-lines, BBKS power
    shape, k_F = 6.5 / Mpc): eight sampled sight-lines, among them two sharing
    a row, against the oracle's plane-by-plane path on the same modes."""
    import torch
    from synth import fields
    w = fields.field_synthesis_workload(device="cuda:0")
    print(f"field synthesis: {w.name}", flush=True)
    b, v = _run(w.modes, w.pk, w.dk, w.amp, w.box, w.k_F, w.E_plus, w.sx, w.sy)
    rows = {}
    for i, y in enumerate(w.sy):
        rows.setdefault(int(y), []).append(i)
    shared = next(r for r in rows.values() if len(r) >= 2)[:2]
    pick = np.unique(np.concatenate([[0, 1, len(w.sx) - 1, 1000, 3333, 5000], shared]))
    modes = w.modes.cpu().numpy()
    del w.modes
    torch.cuda.empty_cache()
    rb, rv = FS.skewer_fields_planes(modes, w.pk, w.dk, w.amp, w.box, w.k_F, w.E_plus,
                                     w.sx[pick], w.sy[pick])
    _assert_close("delta_b (sampled)", b[pick], rb)
    _assert_close("v_z (sampled)", v[pick], rv)
