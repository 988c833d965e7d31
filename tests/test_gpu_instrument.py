"""GPU parity of the instrument model (line-spread convolution, resampling,
noise) and of its adjoint against the FP64 oracle, through the C ABI.

Bar: |F_obs_gpu - F_obs_ref| <= 1e-6 (the flux tolerance; the kernel works in
FP64 and rounds once to FP32, so about 6e-8 is expected), and for the adjoint
||g_gpu - g_ref||_inf <= 1e-6 ||g_ref||_inf."""
import numpy as np
import pytest

from gpu_util import F_ABS, to_dev
from oracle import oracle as O
from synth import fields

pytestmark = pytest.mark.gpu

G_INS = 1e-6


def kms(angstrom):
    return O.angstrom_to_kms(angstrom, fields.REDSHIFT)


def n_bins(lens, dvs, bin_kms, path_kms=None):
    out = []
    for n, dv in zip(lens, dvs):
        L = n * dv if path_kms is None else min(n * dv, path_kms)
        out.append(int(L // bin_kms) if n else 0)
    return out


def offs(lens):
    return np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)


def gpu_instrument(F, dv, off, oo, fwhm, bin_kms, v0=0.0, noise=None, sigma=0.0, k=6.0):
    import torch
    from paper_1105_4747_amd import lyaf as L
    out = torch.full((int(oo[-1]),), float("nan"), device="cuda:0", dtype=torch.float32)
    L.instrument(to_dev(np.asarray(F, np.float32)), to_dev(np.asarray(dv, np.float32)), off, oo,
                 out, fwhm, bin_kms, v0, None if noise is None else to_dev(noise), sigma, k)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def gpu_instrument_bwd(g, dv, off, oo, fwhm, bin_kms, v0=0.0, k=6.0):
    import torch
    from paper_1105_4747_amd import lyaf as L
    out = torch.full((int(off[-1]),), float("nan"), device="cuda:0", dtype=torch.float32)
    L.instrument_backward(to_dev(np.asarray(g, np.float32)), to_dev(np.asarray(dv, np.float32)),
                          off, oo, out, fwhm, bin_kms, v0, k)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


# name: (skewer lengths, dv per skewer, FWHM km/s, bin km/s, v_start, window_k, path)
CASES = {
    "high-res": ([1024, 3000, 40, 0, 777], [2.0, 2.0, 2.0, 2.0, 4.0], 7.0, None, 0.0, 6.0, None),
    "boss": ([4096, 2000, 513], [18.3, 18.3, 18.3], None, None, 0.0, 6.0, "lya-lyb"),
    "sdss": ([4096, 1500], [2.0, 3.0], 170.0, None, -250.0, 6.0, None),
    "bins-at-width-limit": ([5000, 2600], [1.0, 1.0], 224.0, 252.0, -123.0, 6.0, None),
    "sub-pixel-bins": ([700, 333], [4.0, 4.0], 7.0, None, 55.5, 6.0, None),
    "whole-box-even-odd": ([40, 41, 300], [2.0, 3.0, 1.0], 400.0, 5.0, -1e4, 6.0, None),
    "window-k-zero": ([600, 64], [2.0, 2.0], 170.0, 61.65, 10.0, 0.0, None),
    "taps-beyond-a-block": ([2500], [0.5], 224.0, 30.0, 3.0, 6.0, None),
    "no-convolution": ([300, 0, 90], [2.0, 2.0, 2.0], 0.0, 4.0, -1.0, 6.0, None),
    # more than 4096 bins on one skewer: the adjoint reads the bin gradients from
    # memory instead of its LDS copy
    "many-bins": ([9000, 500], [2.0, 2.0], 7.0, 3.0826, 0.0, 6.0, None),
    # boxes shorter than one thread's row of eight staged pixels (the row wraps
    # around the box more than once)
    "tiny-boxes": ([3, 5, 7, 1], [2.0, 2.0, 2.0, 2.0], 3.0, 1.5, -0.7, 6.0, None),
    # 4096 bins (the most the per-skewer adjoint holds in LDS) and 4097 (the
    # per-tile adjoint), with a bin edge on every other pixel edge
    "bins-at-the-lds-limit": ([8192, 8194], [1.0, 1.0], 7.0, 2.0, -3.0, 6.0, None),
    # short taps on short boxes (3 taps on 9 and 13 pixels; the 2-pixel box
    # takes the whole-box form), bins starting several boxes away
    "short-taps-short-boxes": ([9, 13, 2], [2.0, 2.0, 2.0], 1.0, 1.5, -47.3, 6.0, None),
}


def case(name, seed):
    lens, dvs, fwhm, bin_kms, v0, k, path = CASES[name]
    if name == "high-res":
        bin_kms = kms(fields.INSTRUMENT_HIGH_RES["bin_angstrom"])
    if name == "boss":
        fwhm = kms(fields.INSTRUMENT_BOSS["fwhm_angstrom"])
        bin_kms = kms(fields.INSTRUMENT_BOSS["bin_angstrom"])
    if name == "sdss":
        bin_kms = kms(fields.INSTRUMENT_SDSS["bin_angstrom"])
    if name == "sub-pixel-bins":
        bin_kms = kms(fields.INSTRUMENT_HIGH_RES["bin_angstrom"])
    path_kms = O.lya_lyb_path_kms(fields.INSTRUMENT_BOSS["proximity_kms"]) if path else None
    off = offs(lens)
    oo = offs(n_bins(lens, dvs, bin_kms, path_kms))
    rng = np.random.default_rng(seed)
    F = np.exp(-rng.exponential(1.0, off[-1])).astype(np.float32)  # flux in (0, 1]
    return F, np.asarray(dvs, np.float32), off, oo, fwhm, bin_kms, v0, k


@pytest.mark.parametrize("name", sorted(CASES))
def test_instrument_matches_oracle(name):
    F, dv, off, oo, fwhm, bin_kms, v0, k = case(name, 3)
    print(f"case: instrument {name} P={off[-1]} P_out={oo[-1]}", flush=True)
    snr = 50.0
    eps = fields.noise_draws(int(oo[-1]), 9)
    got = gpu_instrument(F, dv, off, oo, fwhm, bin_kms, v0, eps, 1.0 / snr, k)
    want = O.instrument(F.astype(np.float64), off, dv.astype(np.float64), oo, fwhm, bin_kms, v0,
                        eps.astype(np.float64), 1.0 / snr)
    err = float(np.max(np.abs(got - want))) if want.size else 0.0
    assert np.all(np.isfinite(got))
    assert err <= F_ABS, f"{name}: max |dF_obs| {err:.3g}"


@pytest.mark.parametrize("name", sorted(CASES))
def test_instrument_backward_matches_oracle(name):
    F, dv, off, oo, fwhm, bin_kms, v0, k = case(name, 4)
    print(f"case: instrument backward {name} P={off[-1]} P_out={oo[-1]}", flush=True)
    g = np.random.default_rng(5).standard_normal(int(oo[-1])).astype(np.float32)
    got = gpu_instrument_bwd(g, dv, off, oo, fwhm, bin_kms, v0, k)
    want = O.instrument_backward(g.astype(np.float64), off, dv.astype(np.float64), oo, fwhm,
                                 bin_kms, v0)
    assert np.all(np.isfinite(got))
    scale = max(float(np.max(np.abs(want))), 1e-30) if want.size else 1.0
    assert float(np.max(np.abs(got - want), initial=0.0)) <= G_INS * scale


def test_instrument_autograd_and_noise_independence():
    import torch
    from paper_1105_4747_amd import lyaf as L
    F, dv, off, oo, fwhm, bin_kms, v0, k = case("sdss", 6)
    print("case: instrument autograd sdss", flush=True)
    Ft = to_dev(F).requires_grad_(True)
    w = np.random.default_rng(7).standard_normal(int(oo[-1])).astype(np.float32)
    eps = to_dev(fields.noise_draws(int(oo[-1]), 8))
    obs = L.observe(Ft, to_dev(dv), off, oo, fwhm, bin_kms, v0, eps, 0.2, k)
    (obs * to_dev(w)).sum().backward()
    want = O.instrument_backward(w.astype(np.float64), off, dv.astype(np.float64), oo, fwhm,
                                 bin_kms, v0)
    got = Ft.grad.detach().cpu().numpy().astype(np.float64)
    assert float(np.max(np.abs(got - want))) <= G_INS * float(np.max(np.abs(want)))


def test_instrument_domain_status_and_other_skewers_unaffected():
    from paper_1105_4747_amd import lyaf as L
    lens, dvs = [500, 500, 500], np.array([2.0, -1.0, 2.0], np.float32)
    off = offs(lens)
    oo = offs([100, 100, 100])
    F = np.random.default_rng(1).random(off[-1]).astype(np.float32)
    print("case: instrument domain (dv <= 0 on skewer 1)", flush=True)
    L.status_read()
    got = gpu_instrument(F, dvs, off, oo, 7.0, 3.0)
    assert L.status_read() & L.STATUS_DOMAIN
    want = O.instrument(F.astype(np.float64)[np.r_[0:500, 1000:1500]], offs([500, 500]),
                        np.array([2.0, 2.0]), offs([100, 100]), 7.0, 3.0)
    assert float(np.max(np.abs(got[np.r_[0:100, 200:300]] - want))) <= F_ABS
    # bins longer than the box
    print("case: instrument domain (bins longer than the box)", flush=True)
    gpu_instrument(F[:500], np.array([2.0], np.float32), offs([500]), offs([400]), 7.0, 3.0)
    assert L.status_read() & L.STATUS_DOMAIN
    # a clean call leaves the status clear
    gpu_instrument(F[:500], np.array([2.0], np.float32), offs([500]), offs([300]), 7.0, 3.0)
    assert L.status_read() == 0


def _sampled(w, settings, path_kms, n_sample, seed):
    """The instrument on every skewer of a workload's shape (a seeded synthetic
    flux stands in for its forward flux); sampled skewers against the oracle."""
    import torch
    from paper_1105_4747_amd import lyaf as L
    lens = np.diff(w.offsets)
    Fh = fields.synthetic_flux(lens, seed)
    F = to_dev(Fh)
    fwhm, bin_kms, sigma = settings
    oo = offs(n_bins(lens, w.dv, bin_kms, path_kms))
    eps = fields.noise_draws(int(oo[-1]), seed)
    out = torch.empty(int(oo[-1]), device="cuda:0", dtype=torch.float32)
    L.instrument(F, to_dev(w.dv), w.offsets, oo, out, fwhm, bin_kms, 0.0, to_dev(eps), sigma, 6.0)
    torch.cuda.synchronize()
    assert L.status_read() == 0
    got = out.cpu().numpy().astype(np.float64)
    pick = np.sort(np.random.default_rng(seed).choice(w.n_skewers, n_sample, replace=False))
    for s in pick:
        a, b = int(w.offsets[s]), int(w.offsets[s + 1])
        ref = O.instrument(Fh[a:b].astype(np.float64), offs([b - a]), float(w.dv[s]),
                           offs([oo[s + 1] - oo[s]]), fwhm, bin_kms, 0.0,
                           eps[oo[s]:oo[s + 1]].astype(np.float64), sigma)
        err = float(np.max(np.abs(got[oo[s]:oo[s + 1]] - ref)))
        assert err <= F_ABS, f"skewer {s}: max |dF_obs| {err:.3g}"


@pytest.mark.slow
def test_high_resolution_on_config2_sampled():
    w = fields.config2()
    hr = fields.INSTRUMENT_HIGH_RES
    print("case: instrument high-res on C2, 12 sampled skewers", flush=True)
    _sampled(w, (hr["fwhm_kms"], kms(hr["bin_angstrom"]), 1.0 / hr["snr"]), None, 12, 21)


@pytest.mark.slow
def test_boss_on_gpc_sampled():
    w = fields.gpc_lowres()
    bo = fields.INSTRUMENT_BOSS
    path = O.lya_lyb_path_kms(bo["proximity_kms"])
    print("case: instrument BOSS on the Gpc box, 12 sampled skewers", flush=True)
    _sampled(w, (kms(bo["fwhm_angstrom"]), kms(bo["bin_angstrom"]), 1.0 / bo["snr"]), path, 12,
             22)
