"""GPU parity of the flux statistics (Section 4) against the FP64 oracle,
through the C ABI.

Flux PDF: the counts are integers decided in the same precision on both sides
(FP64 floor((F + 0.025) * 20) on the exact FP32 input), so they must agree
exactly.  Power spectrum: the library transforms in FP64 and rounds each P(k_m)
once to FP32, so |P_gpu - P_ref| <= 1e-6 P_ref + 1e-12 max_m P_ref per skewer."""
import numpy as np
import pytest

from gpu_util import to_dev
from oracle import flux_stats as FS
from oracle import oracle as O
from synth import fields

pytestmark = pytest.mark.gpu

P_REL, P_FLOOR = 1e-6, 1e-12


def gpu_pdf(F):
    import torch
    from paper_1105_4747_amd import lyaf as L
    counts = torch.full((L.PDF_SLOTS,), -1, device="cuda:0", dtype=torch.int64)
    L.flux_pdf(to_dev(np.asarray(F, np.float32)) if not hasattr(F, "data_ptr") else F, counts)
    torch.cuda.synchronize()
    return counts.cpu().numpy()


def gpu_power(F, dv, offsets, mean_F):
    import torch
    from paper_1105_4747_amd import lyaf as L
    mo = L.mode_offsets(offsets)
    out = torch.full((int(mo[-1]),), float("nan"), device="cuda:0", dtype=torch.float32)
    Ft = to_dev(np.asarray(F, np.float32)) if not hasattr(F, "data_ptr") else F
    L.flux_power(Ft, to_dev(np.asarray(dv, np.float32)), offsets, mean_F, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def assert_power_close(got, want, offsets, what):
    mo = FS.mode_offsets(offsets)
    assert np.all(np.isfinite(got)), what
    for s in range(len(offsets) - 1):
        g, w = got[mo[s]:mo[s + 1]], want[mo[s]:mo[s + 1]]
        tol = P_REL * np.abs(w) + P_FLOOR * np.max(np.abs(w))
        bad = np.abs(g - w) > tol
        assert not bad.any(), f"{what}: skewer {s}, {bad.sum()} modes off, worst " \
                              f"{np.max(np.abs(g - w) / np.maximum(tol, 1e-300)):.3g} x tol"


def c1_flux():
    """The oracle's F of C1 (full sum, mean-flux rescale), as float32."""
    w = fields.config1()
    raw = O.tau(w.delta, w.vpec, w.dv, w.T0, w.gamma, offsets=w.offsets, tau_ref=w.tau_ref,
                delta_pivot=w.delta_pivot)
    _, F, _ = O.normalise(raw, w.target_F)
    return w, F.astype(np.float32)


def test_pdf_of_the_c1_flux_and_its_noisy_observation():
    w, F = c1_flux()
    print("case: flux PDF of C1 F", flush=True)
    assert np.array_equal(gpu_pdf(F), FS.flux_pdf(F))
    # a BOSS-like noisy observation (S/N 5) of it, by the oracle: values below 0
    # and above 1
    oo = np.arange(w.n_skewers + 1, dtype=np.int64) * 30
    eps = fields.noise_draws(int(oo[-1]), 3).astype(np.float64)
    obs = O.instrument(F.astype(np.float64), w.offsets, w.dv.astype(np.float64), oo, 170.0, 61.65,
                       0.0, eps, 0.2).astype(np.float32)
    print("case: flux PDF of a noisy observation", flush=True)
    want = FS.flux_pdf(obs)
    assert want[FS.PDF_BELOW] > 0 and want[FS.PDF_ABOVE] > 0
    assert np.array_equal(gpu_pdf(obs), want)


def test_pdf_at_bin_edges_and_special_values():
    edges = (-0.025 + 0.05 * np.arange(22)).astype(np.float32)
    vals = np.concatenate([edges, np.nextafter(edges, np.float32(-1)), np.nextafter(edges, np.float32(2)),
                           np.array([np.nan, np.inf, -np.inf, 0.0, 1.0, -0.0], np.float32)])
    vals = np.tile(vals, 3000).astype(np.float32)  # enough for several workgroups
    print(f"case: flux PDF edges n={vals.size}", flush=True)
    got = gpu_pdf(vals)
    want = FS.flux_pdf(vals)
    assert np.array_equal(got, want), (got, want)
    assert got.sum() == vals.size


def test_pdf_of_nothing_and_of_one_value():
    import torch
    print("case: flux PDF empty and single", flush=True)
    got = gpu_pdf(torch.empty(0, device="cuda:0", dtype=torch.float32))
    assert np.array_equal(got, np.zeros(24, np.int64))
    got = gpu_pdf(np.array([0.51], np.float32))
    assert got[10] == 1 and got.sum() == 1


@pytest.mark.slow
def test_pdf_at_full_size():
    F = fields.synthetic_flux(np.full(4096, 4096), 12)
    print("case: flux PDF of a 4096 x 4096 synthetic flux (16.8M px)", flush=True)
    assert np.array_equal(gpu_pdf(F), FS.flux_pdf(F))


@pytest.mark.parametrize("lens", [[1024] * 8, [2, 4, 8, 16, 512, 4096, 8192, 2]])
def test_power_matches_oracle(lens):
    rng = np.random.default_rng(len(lens))
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    F = np.exp(-rng.exponential(0.5, off[-1])).astype(np.float32)
    dv = rng.uniform(1.0, 20.0, len(lens)).astype(np.float32)
    print(f"case: flux power lens={lens}", flush=True)
    got = gpu_power(F, dv, off, 0.72)
    want, _ = FS.flux_power(F.astype(np.float64), off, dv.astype(np.float64), 0.72)
    assert_power_close(got, want, off, f"lens {lens}")


def test_power_of_the_c1_flux():
    w, F = c1_flux()
    print("case: flux power of C1 F", flush=True)
    got = gpu_power(F, w.dv, w.offsets, w.target_F)
    want, _ = FS.flux_power(F.astype(np.float64), w.offsets, w.dv.astype(np.float64), w.target_F)
    assert_power_close(got, want, w.offsets, "C1")


def test_power_domain_status():
    from paper_1105_4747_amd import lyaf as L
    off = np.array([0, 64, 128], np.int64)
    F = np.random.default_rng(0).random(128).astype(np.float32)
    print("case: flux power with dv <= 0", flush=True)
    L.status_read()
    got = gpu_power(F, np.array([2.0, 0.0], np.float32), off, 0.8)
    assert L.status_read() & L.STATUS_DOMAIN
    want, _ = FS.flux_power(F[:64].astype(np.float64), [0, 64], 2.0, 0.8)
    assert_power_close(got[:33], want, [0, 64], "good skewer")


@pytest.mark.slow
@pytest.mark.parametrize("name", ["config2", "gpc_lowres"])
def test_power_full_size_sampled(name):
    w = getattr(fields, name)()
    Fh = fields.synthetic_flux(np.diff(w.offsets), 13)
    print(f"case: flux power of a synthetic flux of {w.name}'s shape, 16 sampled skewers",
          flush=True)
    got = gpu_power(Fh, w.dv, w.offsets, w.target_F)
    mo = FS.mode_offsets(w.offsets)
    for s in np.sort(np.random.default_rng(7).choice(w.n_skewers, 16, replace=False)):
        a, b = int(w.offsets[s]), int(w.offsets[s + 1])
        want, _ = FS.flux_power(Fh[a:b].astype(np.float64), [0, b - a], float(w.dv[s]),
                                w.target_F)
        assert_power_close(got[mo[s]:mo[s + 1]], want, [0, b - a], f"{w.name} skewer {s}")


def test_power_unaligned_flux_and_short_skewers():
    """Flux that starts 4 bytes past an 8-byte boundary (the library then reads
    it value by value) and skewers of every power-of-two length from 2 to 8192,
    whose offsets leave the later skewers at odd multiples of 2 values."""
    import torch
    lens = [2 ** k for k in range(1, 14)] + [2, 4, 8]
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    rng = np.random.default_rng(17)
    F = np.exp(-rng.exponential(0.4, int(offsets[-1]))).astype(np.float32)
    dv = rng.uniform(1.0, 4.0, len(lens)).astype(np.float32)
    want, _ = FS.flux_power(F.astype(np.float64), offsets, dv.astype(np.float64), 0.7)
    for shift in (0, 1):
        print(f"case: power, {len(lens)} skewers of 2..8192 px, flux shifted by {shift} value",
              flush=True)
        base = torch.zeros(int(offsets[-1]) + 2, device="cuda:0", dtype=torch.float32)
        base[shift:shift + int(offsets[-1])] = to_dev(F)
        got = gpu_power(base[shift:shift + int(offsets[-1])], dv, offsets, 0.7)
        assert_power_close(got, want, offsets, f"shift {shift}")


def test_pdf_of_unaligned_flux():
    """Flux that starts 0-3 values past a 16-byte boundary, with lengths that
    leave a ragged end: the library reads whole 16-byte groups in between and
    the values at either end one by one."""
    import torch
    rng = np.random.default_rng(23)
    F = rng.uniform(-0.1, 1.1, 50003).astype(np.float32)
    F[::97] = np.nan
    for shift in range(4):
        for n in (0, 1, 5, 4099, 50003 - shift):
            print(f"case: pdf of {n} values at offset {shift}", flush=True)
            base = torch.zeros(50008, device="cuda:0", dtype=torch.float32)
            base[shift:shift + n] = to_dev(F[:n])
            got = gpu_pdf(base[shift:shift + n])
            assert np.array_equal(got, FS.flux_pdf(F[:n])), (shift, n)
