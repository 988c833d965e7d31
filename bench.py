#!/usr/bin/env python3
"""Throughput of the Lyman-alpha optical-depth hot path on one MI355X.

One step = the whole path over the 4096 x 4096 workload (4096 skewers of 4096
pixels, dv = 2 km/s, sigma_lnDelta = 1.2, T0 = 2e4 K, gamma = 1.3, window
+-6 b, target <F> = 0.75; synthetic lognormal fields, seed 2) with the inputs
resident in HBM: one replay of a tuned plan, i.e. the hipGraph of the reach
pass, the windowed tau kernel, the FP64 mean-flux root-find passes and
tau' = A tau, F = exp(-tau').

Prints one JSON line.  ``value`` is skewer-pixels per second of tau + F.
``roofline`` describes the dominant kernel, the windowed tau kernel: the
algorithmic pairs inside the +-k b window (counted exactly from the inputs)
times 5 FP32 flops per pair (the offset FMA, the scaling, the square and the
accumulating FMA; the exp2 is not counted), divided by the kernel's average
duration (HIP events the library records around that launch alone, on its
stream), against the FP32 vector peak of 157.3 TFLOP/s.  Beside it: the pair
rate against the ceiling of the direct form, min(FMA rate / 3, exp2 rate),
both measured on the device in the same run (libpeaks).  ``error`` states the
FP32 results against the FP64 oracle on the CPU-baseline sample.
``cpu_baseline`` is the FP64 oracle (full sum + root-find) on a bounded sample
of the same workload on the host cores.  ``detail`` holds the other
workloads: the ragged 20,000-skewer batch, the 512 x 512 x 4096 box, the
adjoint, the instrument model and the flux statistics.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("skewer-pixels/sec of τ+F at stated FP32 error vs FP64 oracle; roofline %")
FP32_PEAK_TFLOPS = 157.3      # 256 CU x 4 SIMD x 16 lanes x 2 (packed) x 2 (FMA) x 2.4 GHz
# The library is built without packed FP32 instructions, so one FP32 op issues
# per lane and cycle: 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz.
FP32_UNPACKED_TFLOPS = 78.6
# algorithmic FP32 flops of one source-target pair: the offset FMA (counted
# as 1 with the scaling multiply, 1), the square (1) and the accumulating FMA
# (2); the exp2 is a transcendental, not a flop
FLOPS_PER_PAIR = 5
HBM_PEAK_GBPS = 8000.0
TAU_TOL_REL, TAU_TOL_FLOOR, F_TOL_ABS = 1e-5, 1e-3, 1e-6


def algorithmic_pairs(w) -> float:
    """sum over sources j of #{i : |(i - j) dv - v_j| < k b_j}, clamped to N,
    with b_j from the T-rho relation (FP64, host; a box held on the GPU is
    copied over in chunks of skewers)."""
    kB, mH = 1.380649e-16, 1.6735575e-24
    total = 0.0
    lens = np.diff(w.offsets)
    on_device = not isinstance(w.delta, np.ndarray)
    step = 4096 if on_device else 256
    for s0 in range(0, w.n_skewers, step):
        s1 = min(w.n_skewers, s0 + step)
        a, b = int(w.offsets[s0]), int(w.offsets[s1])
        if on_device:
            d = w.delta[a:b].cpu().numpy().astype(np.float64)
            v = w.vpec[a:b].cpu().numpy().astype(np.float64)
        else:
            d = w.delta[a:b].astype(np.float64)
            v = w.vpec[a:b].astype(np.float64)
        sk = np.repeat(np.arange(s0, s1), lens[s0:s1])
        dv, T0, gm = (w.dv[sk].astype(np.float64), w.T0[sk].astype(np.float64),
                      w.gamma[sk].astype(np.float64))
        D = np.minimum(d, w.delta_pivot)
        with np.errstate(divide="ignore", invalid="ignore"):
            T = T0 * np.where(D > 0, D, 1.0) ** (gm - 1)
        bj = np.sqrt(2 * kB * T / mH) / 1e5
        h = w.window_k * bj / dv
        c = v / dv
        # count integers m with c - h < m < c + h
        cnt = np.ceil(c + h) - np.floor(c - h) - 1
        cnt = np.minimum(np.maximum(cnt, 0), lens[sk])
        total += float(np.where(d > 0, cnt, 0).sum())
    return total


def adjoint_section(L, torch, dev, fields, timed, reps, peak):
    """The hand-written adjoint on the 4096 x 2048 workload: lyaf_tau_backward
    (reach pass, adjoint pair kernel, per-skewer FP64 sums) for a random
    cotangent, and the forward tau stage for comparison; HIP events."""
    w = fields.config5()
    print(f"bench: adjoint {w.name}", file=sys.stderr, flush=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    d = [t(x) for x in (w.delta, w.vpec, w.dv, w.T0, w.gamma)]
    P = w.n_pix
    raw = torch.empty(P, device=dev, dtype=torch.float32)
    g = torch.randn(P, device=dev, generator=torch.Generator(device=dev).manual_seed(5))
    gd, gv = torch.empty_like(raw), torch.empty_like(raw)
    gT = torch.empty(w.n_skewers, device=dev, dtype=torch.float64)
    gg = torch.empty_like(gT)
    t_fwd = timed(lambda: L.tau(*d, w.offsets, raw, window_k=w.window_k), reps)
    t_bwd = timed(lambda: L.tau_backward(*d, w.offsets, g, gd, gv, gT, gg,
                                         window_k=w.window_k), reps)
    pairs = algorithmic_pairs(w)
    # one interleaved autograd step: tau', F and A forward (implicit-A rescale),
    # the loss sum (F - F_t)^2, and its gradients for Delta, v, T0 and gamma
    dd = [x.clone().requires_grad_(i != 2) for i, x in enumerate(d)]  # all but dv
    F_t = torch.rand(P, device=dev, generator=torch.Generator(device=dev).manual_seed(6))

    def step():
        for x in dd:
            x.grad = None
        _, F, _ = L.tau_flux(dd[0], dd[1], dd[3], dd[4], dd[2], w.offsets, w.target_F,
                             tau_ref=w.tau_ref, delta_pivot=w.delta_pivot, window_k=w.window_k)
        ((F - F_t) ** 2).sum().backward()
    t_step = timed(step, reps)
    out = {"workload": w.name, "n_pix": P, "tau_backward_ms": round(t_bwd * 1e3, 4),
           "tau_forward_ms": round(t_fwd * 1e3, 4), "pairs_per_px": round(pairs / P, 2),
           "adjoint_pair_rate_per_s": pairs / t_bwd, "px_per_s": P / t_bwd,
           "autograd_step_ms": round(t_step * 1e3, 4),
           "autograd_step": "tau_flux forward + loss + backward (Delta, v, T0, gamma)"}
    return out


FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64 (AMD-published)
HBM_PEAK_GBS = 8000.0


def instrument_traffic(case, direction="per_case"):
    """HBM bytes per instrument forward ("per_case") or backward
    ("backward_per_case") launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE record, or None when the kernel sources changed since the
    counters were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "instrument_traffic.json")))
    except OSError:
        return None
    h = hashlib.sha256()
    for f in ("lyaf_instrument.hip", "lyaf_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1105_4747_amd", "csrc", f), "rb").read())
    if h.hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    ent = rec.get(direction, {}).get(case)
    return None if ent is None else ent["traffic_bytes_per_launch"]


def instrument_case(L, torch, dev, fields, timed, reps, case, name, F, dvt, w, settings,
                    path_kms):
    """Time lyaf_instrument (and its backward) on the flux F of workload w."""
    fwhm, bin_kms, sigma = settings
    lens = np.diff(w.offsets)
    n_out = []
    covered = 0
    for n, dv in zip(lens, w.dv):
        L_kms = n * float(dv) if path_kms is None else min(n * float(dv), path_kms)
        k = int(L_kms // bin_kms)
        n_out.append(k)
        covered += min(int(n), int(np.ceil(k * bin_kms / float(dv))) + 1)
    oo = np.concatenate([[0], np.cumsum(n_out)]).astype(np.int64)
    Po = int(oo[-1])
    eps = torch.from_numpy(fields.noise_draws(Po, 31)).to(dev)
    obs = torch.empty(Po, device=dev, dtype=torch.float32)
    gF = torch.empty_like(F)
    g = torch.from_numpy(fields.noise_draws(Po, 32)).to(dev)
    run = lambda: L.instrument(F, dvt, w.offsets, oo, obs, fwhm, bin_kms, 0.0, eps, sigma, 6.0)
    t_fwd = timed(run, reps)
    t_bwd = timed(lambda: L.instrument_backward(g, dvt, w.offsets, oo, gF, fwhm, bin_kms, 0.0,
                                                6.0), reps)
    if L.status_read() != 0:
        raise RuntimeError(f"device status set in the instrument case {name}")
    # algorithmic work: taps within +-6 b_L per covered pixel (FMA = 2 flops);
    # bytes: F read once, noise read and F_obs written per bin
    bL = fwhm / (2.0 * np.sqrt(np.log(2.0)))
    taps = 2 * int(np.floor(6.0 * bL / float(w.dv[0]))) + 1
    flops = 2.0 * taps * covered
    nbytes = 4.0 * covered + 8.0 * Po
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_fp64 = flops / (FP64_PEAK_TFLOPS * 1e12)
    if t_fp64 >= t_hbm:
        roof = {"bound": "fp64", "achieved": round(flops / t_fwd / 1e12, 3),
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": round(nbytes / t_fwd / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["traffic"] = instrument_traffic(case)
    roof["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE)"
    return {"workload": name, "fwhm_kms": round(fwhm, 3), "bin_kms": round(bin_kms, 4),
            "noise_sigma": sigma, "n_pix": int(w.n_pix), "covered_px": covered, "n_bins": Po,
            "taps": taps, "forward_ms": round(t_fwd * 1e3, 4), "backward_ms": round(t_bwd * 1e3, 4),
            "px_per_s": covered / t_fwd, "bins_per_s": Po / t_fwd,
            "algorithmic_bytes": int(nbytes), "algorithmic_flops": flops,
            "hbm_GBs": round(nbytes / t_fwd / 1e9, 1),
            "fp64_TFLOPs": round(flops / t_fwd / 1e12, 3), "roofline": roof,
            "kernel": "instrument_kernel",
            "backward_kernel": "instrument_backward_skewer_kernel (skewers of at most 4096 bins)",
            "backward_traffic": instrument_traffic(case, "backward_per_case")}


def instrument_section(L, torch, dev, fields, timed, reps, F_c2, dvt_c2, w_c2):
    """The instrument model (Sections 3.1, 3.2): the paper's high-resolution
    setting on the 4096 x 4096 workload's flux, and its BOSS-like setting on the
    Gpc box's flux (forward tau and mean-flux rescale first)."""
    z = fields.REDSHIFT
    hr, bo = fields.INSTRUMENT_HIGH_RES, fields.INSTRUMENT_BOSS
    out = {}
    print("bench: instrument high-res", file=sys.stderr, flush=True)
    out["high_res"] = instrument_case(
        L, torch, dev, fields, timed, reps, "high_res", w_c2.name, F_c2, dvt_c2, w_c2,
        (hr["fwhm_kms"], L.angstrom_to_kms(hr["bin_angstrom"], z), 1.0 / hr["snr"]), None)
    w = fields.gpc_lowres()
    print(f"bench: instrument BOSS-like on {w.name}", file=sys.stderr, flush=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    d = [t(x) for x in (w.delta, w.vpec, w.dv, w.T0, w.gamma)]
    raw = torch.empty(w.n_pix, device=dev, dtype=torch.float32)
    F = torch.empty_like(raw)
    A = torch.empty((), device=dev, dtype=torch.float64)
    L.tau(*d, w.offsets, raw, tau_ref=w.tau_ref, delta_pivot=w.delta_pivot, window_k=w.window_k)
    L.normalise_mean_flux(raw, F, w.target_F, A)
    out["boss"] = instrument_case(
        L, torch, dev, fields, timed, reps, "boss", w.name, F, d[2], w,
        (L.angstrom_to_kms(bo["fwhm_angstrom"], z), L.angstrom_to_kms(bo["bin_angstrom"], z),
         1.0 / bo["snr"]), L.lya_lyb_path_kms(bo["proximity_kms"]))
    return out


def stats_section(L, torch, dev, timed, reps, F, dvt, w):
    """The flux statistics of Section 4 on the 4096 x 4096 workload's flux: the
    21-bin flux PDF (lyaf_flux_pdf) and the per-skewer 1D flux power spectrum
    (lyaf_flux_power), HIP events."""
    P = int(F.numel())
    counts = torch.empty(L.PDF_SLOTS, device=dev, dtype=torch.int64)
    t_pdf = timed(lambda: L.flux_pdf(F, counts), reps)
    mo = L.mode_offsets(w.offsets)
    power = torch.empty(int(mo[-1]), device=dev, dtype=torch.float32)
    t_ps = timed(lambda: L.flux_power(F, dvt, w.offsets, w.target_F, power), reps)
    if L.status_read() != 0:
        raise RuntimeError("device status set in the statistics section")
    pdf_bytes = 4.0 * P
    # power: 4 B per pixel in, 4 B per mode out; FP64 work of an N/2-point
    # complex FFT per skewer (5 M log2 M flops) plus ~20 flops per mode
    lens = np.diff(w.offsets)
    ps_bytes = 4.0 * P + 4.0 * float(mo[-1])
    ps_flops = float(sum(5.0 * (n // 2) * np.log2(max(n // 2, 1)) + 20.0 * (n // 2 + 1)
                         for n in lens))
    t_hbm, t_fp64 = ps_bytes / (HBM_PEAK_GBS * 1e9), ps_flops / (FP64_PEAK_TFLOPS * 1e12)
    ps_roof = ({"bound": "hbm", "achieved": round(ps_bytes / t_ps / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s"} if t_hbm >= t_fp64 else
               {"bound": "fp64", "achieved": round(ps_flops / t_ps / 1e12, 3),
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"})
    ps_roof["frac"] = round(ps_roof["achieved"] / ps_roof["peak"], 4)
    pdf_gbs = pdf_bytes / t_pdf / 1e9
    return {"workload": w.name, "n_pix": P,
            "flux_pdf": {"ms": round(t_pdf * 1e3, 4), "px_per_s": P / t_pdf,
                         "algorithmic_bytes": int(pdf_bytes),
                         "roofline": {"bound": "hbm", "achieved": round(pdf_gbs, 1),
                                      "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                      "frac": round(pdf_gbs / HBM_PEAK_GBS, 4)},
                         "kernel": "flux_pdf_kernel + flux_pdf_sum_kernel"},
            "flux_power": {"ms": round(t_ps * 1e3, 4), "px_per_s": P / t_ps,
                           "modes": int(mo[-1]), "algorithmic_bytes": int(ps_bytes),
                           "algorithmic_fp64_flops": ps_flops,
                           "fp64_TFLOPs": round(ps_flops / t_ps / 1e12, 3),
                           "roofline": ps_roof, "kernel": "flux_power_kernel"}}


def _hbm_roof(nbytes, seconds):
    gbs = nbytes / seconds / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def fields_section(L, torch, dev, fields, timed, reps):
    """Skewer-only field synthesis (lyaf_field_skewers, eqs. 1 and 3, Appendix B)
    on a 1024^3 grid with 6,250 sight-lines: the whole call and each of its
    three kernels (HIP events the library records), each kernel against HBM
    with its algorithmic bytes."""
    w = fields.field_synthesis_workload(device=dev)
    print(f"bench: {w.name}", file=sys.stderr, flush=True)
    n, S = w.n, len(w.sx)
    H = n // 2 + 1
    pk = torch.from_numpy(w.pk).to(dev)
    b = torch.empty((S, n), device=dev, dtype=torch.float32)
    v = torch.empty_like(b)
    call = lambda: L.field_skewers(w.modes, pk, w.sx, w.sy, b, v, n, w.box, w.amp, w.k_F,
                                   w.E_plus, w.dk)
    t_call = timed(call, reps)
    t_ky = kernel_seconds(L, call, reps, "field_ky")
    t_kx = kernel_seconds(L, call, reps, "field_kx")
    t_z = kernel_seconds(L, call, reps, "field_z")
    if L.status_read() != 0:
        raise RuntimeError("device status set in the field-synthesis section")
    rows = len(np.unique(w.sy))
    modes = float(n) * n * H
    groups = sum(-(-c // 8) for c in np.unique(w.sy, return_counts=True)[1])
    ky_bytes = 8.0 * modes + 2 * 8.0 * rows * n * H          # modes in, both fields' rows out
    kx_bytes = 2 * 8.0 * groups * n * H + 2 * 16.0 * S * H   # rows in (per group), sums out
    z_bytes = 2 * 16.0 * S * H + 2 * 4.0 * S * n
    kernels = {"field_ky_kernel": (t_ky, ky_bytes), "field_kx_kernel": (t_kx, kx_bytes),
               "field_z_kernel": (t_z, z_bytes)}
    dom = max(kernels, key=lambda k: kernels[k][0])
    return {"workload": w.name, "n": n, "sight_lines": S, "rows_in_use": rows,
            "call_ms": round(t_call * 1e3, 4),
            "sight_line_pixels_per_s": S * n / t_call, "modes_per_s": modes / t_call,
            "kernels": {k: {"ms": round(t * 1e3, 4), "algorithmic_bytes": int(nb),
                            "roofline": _hbm_roof(nb, t)} for k, (t, nb) in kernels.items()},
            "call_minimum_bytes": int(8.0 * modes + 2 * 4.0 * S * n),
            "call_minimum_frac": round(8.0 * modes / t_call / 1e9 / HBM_PEAK_GBS, 4),
            "dominant_kernel": dom, "roofline": {**_hbm_roof(kernels[dom][1], kernels[dom][0]),
                                                 "kernel": dom}}


def power3d_section(L, torch, dev, fields, timed, reps):
    """3D flux power reconstruction of eq. (7) (lyaf_flux_power_3d) from 6,250
    sight-lines of 1024 pixels in a 1024^3 box, shells of the fundamental: the
    whole call (HIP events), against HBM with the bytes of the grid-free method
    (the row sums written and read once, the sight-line spectra, the input)."""
    w = fields.power3d_workload()
    print(f"bench: {w.name}", file=sys.stderr, flush=True)
    n, S = w.n, len(w.sx)
    H = n // 2 + 1
    F = torch.from_numpy(w.F).to(dev)
    nb = int(np.floor(np.sqrt(3) * n / 2)) + 1
    outs = [torch.empty(nb, device=dev, dtype=torch.float64) for _ in range(4)]
    call = lambda: L.flux_power_3d(F, w.mean_F, w.sx, w.sy, n, w.box, nb, *outs,
                                   p_noise=w.p_noise)
    t_call = timed(call, reps)
    t_k = kernel_seconds(L, call, reps, "flux_power_3d")
    if L.status_read() != 0:
        raise RuntimeError("device status set in the 3D power section")
    rows = len(np.unique(w.sy))
    nbytes = 4.0 * S * n + 2 * 16.0 * S * H + 2 * 16.0 * n * rows * H + 8.0 * n * n
    return {"workload": w.name, "n": n, "sight_lines": S, "rows_in_use": rows, "shells": nb,
            "call_ms": round(t_call * 1e3, 4), "kernels_ms": round(t_k * 1e3, 4),
            "modes_per_s": float(n) * n * H / t_call,
            "method_bytes": int(nbytes),
            "roofline": {**_hbm_roof(nbytes, t_k), "kernel": "every kernel of the call"}}


def kernel_seconds(L, fn, reps, name):
    """Average duration (s) of the library's launches recorded under ``name``
    while ``fn`` runs ``reps`` times (HIP events the library records around
    those launches on their stream)."""
    fn()
    L.kernel_timing(True)
    for _ in range(reps):
        fn()
    ms, n = L.kernel_timing_read(name)
    L.kernel_timing(False)
    if n == 0:
        raise RuntimeError(f"no launch recorded under {name}")
    return ms / n * 1e-3


def tau_roofline(pairs, t_kernel, kernel, peak=None):
    """FP32 roofline of the windowed tau kernel: 5 flops per algorithmic pair
    over its average duration, against the packed FP32 peak."""
    ach = pairs * FLOPS_PER_PAIR / t_kernel / 1e12
    out = {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": round(ach / FP32_PEAK_TFLOPS, 4),
           "kernel": kernel, "kernel_ms": round(t_kernel * 1e3, 4),
           "flops_per_pair": FLOPS_PER_PAIR, "pairs_per_launch": pairs,
           "pair_rate_per_s": pairs / t_kernel,
           "unpacked_peak": FP32_UNPACKED_TFLOPS,
           "unpacked_frac": round(ach / FP32_UNPACKED_TFLOPS, 4)}
    if peak is not None:
        out["pair_ceiling_per_s"] = peak["pair_peak_per_s"]
        out["pair_ceiling_frac"] = round(pairs / t_kernel / peak["pair_peak_per_s"], 4)
    return out


def batched_section(L, torch, dev, fields, timed, reps, peak):
    """The ragged 20,000-skewer batch (lengths 512-8192 px, dv 1-4 km/s, T0
    and gamma drawn per skewer): one tuned plan (hipGraph) against the same
    windowed kernel launched once per skewer, and the plain full-sum kernel on
    the first 200 skewers.  The tuner's own median timings of every candidate
    are reported beside the two launch forms of the chosen shape."""
    w = fields.config3()
    print(f"bench: batched {w.name}, P={w.n_pix}", file=sys.stderr, flush=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    delta, vpec, dvt, T0, gamma = t(w.delta), t(w.vpec), t(w.dv), t(w.T0), t(w.gamma)
    P = w.n_pix
    ts = torch.empty(P, device=dev, dtype=torch.float32)
    F = torch.empty_like(ts)
    A = torch.empty((), device=dev, dtype=torch.float64)
    plan = L.Plan(delta, vpec, dvt, T0, gamma, w.offsets, w.target_F, ts, F, A,
                  window_k=w.window_k, autotune=True)
    info = plan.describe()
    t_plan = timed(plan.execute, reps)
    shape = info["shape"]
    pers = info["persistent_grid"] > 0
    fl = L.FLAG_SHAPE(shape) | (L.FLAG_PERSISTENT if pers else 0)
    raw = torch.empty_like(ts)
    tau = lambda flags: L.tau(delta, vpec, dvt, T0, gamma, w.offsets, raw,
                              window_k=w.window_k, flags=flags)
    t_kernel = kernel_seconds(L, lambda: tau(fl), reps, "tau")
    t_grid = kernel_seconds(L, lambda: tau(L.FLAG_SHAPE(shape)), reps, "tau")
    t_pers = kernel_seconds(L, lambda: tau(L.FLAG_SHAPE(shape) | L.FLAG_PERSISTENT), reps, "tau")
    t_per = timed(lambda: tau(L.FLAG_PER_SKEWER | L.FLAG_SHAPE(shape)), 1)
    sub = w.subset(range(200))
    d2 = [t(x) for x in (sub.delta, sub.vpec, sub.dv, sub.T0, sub.gamma)]
    raw2 = torch.empty(sub.n_pix, device=dev, dtype=torch.float32)
    t_plain = timed(lambda: L.tau(*d2, sub.offsets, raw2, window_k=w.window_k,
                                  flags=L.FLAG_PLAIN), 1)
    pairs = algorithmic_pairs(w)
    plan.close()
    return {"workload": w.name, "n_pix": P, "plan": info,
            "plan_step_ms": round(t_plan * 1e3, 4), "px_per_s": P / t_plan,
            "tau_kernel_ms": round(t_kernel * 1e3, 4),
            "tau_kernel_grid_ms": round(t_grid * 1e3, 4),
            "tau_kernel_persistent_ms": round(t_pers * 1e3, 4),
            "chosen_launch": "persistent" if pers else "grid",
            "tau_stage_launch_per_skewer_ms": round(t_per * 1e3, 3),
            "plain_fp32_px_per_s_first200": sub.n_pix / t_plain,
            "pairs_per_px": round(pairs / P, 3),
            "tau_roofline": tau_roofline(pairs, t_kernel,
                                         tau_kernel_name(shape, pers), peak)}


def box_section(L, torch, dev, fields, timed, reps, peak):
    """The 512 x 512 x 4096 box (1.07e9 pixels, 4.3 GB per FP32 array, one
    seeded 3D lognormal field generated on the GPU): one tuned plan replayed
    (tau, global FP64 mean-flux rescale, F), and the windowed kernel's
    roofline."""
    w = fields.config4(device=dev)
    print(f"bench: box {w.name}, P={w.n_pix}", file=sys.stderr, flush=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    dvt, T0, gamma = t(w.dv), t(w.T0), t(w.gamma)
    P = w.n_pix
    ts = torch.empty(P, device=dev, dtype=torch.float32)
    F = torch.empty_like(ts)
    A = torch.empty((), device=dev, dtype=torch.float64)
    plan = L.Plan(w.delta, w.vpec, dvt, T0, gamma, w.offsets, w.target_F, ts, F, A,
                  window_k=w.window_k, autotune=True)
    info = plan.describe()
    t_plan = timed(plan.execute, reps)
    if plan.status() != 0:
        raise RuntimeError("device status set in the box section")
    shape, pers = info["shape"], info["persistent_grid"] > 0
    fl = L.FLAG_SHAPE(shape) | (L.FLAG_PERSISTENT if pers else 0)
    del F
    raw = ts  # reused as the eager tau output
    t_kernel = kernel_seconds(
        L, lambda: L.tau(w.delta, w.vpec, dvt, T0, gamma, w.offsets, raw, window_k=w.window_k,
                         flags=fl), reps, "tau")
    plan.close()
    pairs = algorithmic_pairs(w)
    out = {"workload": w.name, "n_pix": P, "plan": info, "steps": reps,
           "plan_step_ms": round(t_plan * 1e3, 3), "px_per_s": P / t_plan,
           "pairs_per_px": round(pairs / P, 3),
           "tau_roofline": tau_roofline(pairs, t_kernel, tau_kernel_name(shape, pers), peak)}
    del w, ts, raw
    torch.cuda.empty_cache()
    return out


def tau_kernel_name(shape: int, persistent: bool) -> str:
    """Kernel that LYAF_FLAG_SHAPE(shape) launches (as rocprofv3 names it):
    shapes 0, 1, 4 and 5 are the skewed per-lane-run form (4 waves, 2 waves,
    4 waves with the Gaussian recurrence across a lane's 4 targets, the same
    across 8 targets), 2-3 the shared-run form with source streams."""
    suffix = "_persistent_kernel" if persistent else "_kernel"
    return {0: "tau_skew%s<4, false, 4>", 1: "tau_skew%s<2, false, 4>", 2: "tau_window%s<8, 4, 512>",
            3: "tau_window%s<8, 2, 512>", 4: "tau_skew%s<4, true, 4>",
            5: "tau_skew%s<4, true, 8>"}[shape] % suffix


def measured_traffic(shape: int, persistent: bool, workload: str):
    """HBM bytes per windowed tau kernel launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE record, or None when the kernel sources changed
    since the counters were taken (or this shape/launch/workload was not
    counted)."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "tau_kernel_traffic.json")))
    except OSError:
        return None
    h = hashlib.sha256()
    for f in ("lyaf_tau.hip", "lyaf_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1105_4747_amd", "csrc", f), "rb").read())
    if h.hexdigest()[:16] != rec["source_sha256_16"] or persistent or \
            not workload.startswith("C2"):
        return None
    ent = rec["per_shape"].get(str(shape))
    return None if ent is None else ent["traffic_bytes_per_launch"]


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(w, target_seconds=10.0):
    """FP64 oracle on the host: full sum of eq. (6) + mean-flux root-find, on
    the first skewers of the workload, sized to ~target_seconds of wall time.
    Returns the record and the sample with the oracle's raw tau and F (F of
    the sample normalised on its own)."""
    from oracle import oracle as O
    n = 8
    t_run = 0.0
    while True:
        sub = w.subset(range(n))
        t0 = time.perf_counter()
        raw = O.tau(sub.delta, sub.vpec, sub.dv, sub.T0, sub.gamma, offsets=sub.offsets,
                    tau_ref=sub.tau_ref, delta_pivot=sub.delta_pivot)
        _, F, _ = O.normalise(raw, sub.target_F)
        t_run = time.perf_counter() - t0
        if t_run >= target_seconds / 4 or n >= w.n_skewers:
            break
        n = min(w.n_skewers, max(2 * n, int(n * target_seconds / 4 / max(t_run, 1e-3))))
    rec = {"value": sub.n_pix / t_run, "unit": "skewer-pixels/s",
           "cores": O.num_threads(), "cpu_model": cpu_model(), "kind": "oracle",
           "sample": f"first {n} skewers of the workload ({sub.n_pix} px), FP64 full "
                     f"O(N^2) sum + root-find, {t_run:.2f} s"}
    return rec, sub, raw, F


def error_vs_oracle(L, torch, dev, raw_gpu, sub, raw_ref, F_ref):
    """The FP32 results against the FP64 oracle on the CPU-baseline sample:
    raw tau (|err| / (1e-5 max(tau, 1e-3))) and F of the sample, each side
    normalising the sample on its own (|dF| against 1e-6)."""
    g = raw_gpu[:sub.n_pix].clone()
    err = np.abs(g.cpu().numpy().astype(np.float64) - raw_ref)
    tau_ratio = float(np.max(err / (TAU_TOL_REL * np.maximum(raw_ref, TAU_TOL_FLOOR))))
    F = torch.empty_like(g)
    A = torch.empty((), device=dev, dtype=torch.float64)
    L.normalise_mean_flux(g, F, sub.target_F, A)
    dF = float(np.max(np.abs(F.cpu().numpy().astype(np.float64) - F_ref)))
    return {"sample_px": int(sub.n_pix),
            "tau_raw_max_err_over_tol": round(tau_ratio, 4),
            "tau_tol": "1e-5 * max(tau, 1e-3)",
            "F_max_abs_err": dF, "F_tol": F_TOL_ABS,
            "F_max_err_over_tol": round(dF / F_TOL_ABS, 4),
            "F_sample_normalised_on_its_own": True}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-box", action="store_true",
                    help="skip the 512 x 512 x 4096 box (8.6 GB of inputs)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-peaks", action="store_true")
    ap.add_argument("--no-instrument", action="store_true")
    ap.add_argument("--no-stats", action="store_true")
    ap.add_argument("--no-fields", action="store_true")
    ap.add_argument("--no-power3d", action="store_true")
    ap.add_argument("--fields-only", action="store_true",
                    help="only run the field-synthesis section, for profiling")
    ap.add_argument("--power3d-only", action="store_true",
                    help="only run the 3D flux power section, for profiling")
    ap.add_argument("--stats-only", action="store_true",
                    help="only run the flux-statistics section (PDF, power spectrum), for profiling")
    ap.add_argument("--instrument-only", action="store_true",
                    help="only run the instrument section (forward and backward), for profiling")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only run the adjoint section (4096 x 2048), for profiling")
    ap.add_argument("--workload", default="config2", choices=["config2", "config3", "config5"])
    ap.add_argument("--tau-only", action="store_true",
                    help="only run lyaf_tau (reach + windowed kernel) K times, for profiling")
    ap.add_argument("--shape", type=int, default=None,
                    help="windowed-kernel shape for --tau-only (LYAF_FLAG_SHAPE); default: 4, "
                         "the library's own default")
    ap.add_argument("--persistent", action="store_true", help="persistent launch in --tau-only")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB float32 buffer 3 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this path runs on one GPU; --gpus N > 1 is not "
                          "supported (skewers are independent: a batch shards by whole "
                          "skewers, with one all-reduce of the mean-flux sums per "
                          "root-find pass)"}))
        sys.exit(2)

    import torch

    from paper_1105_4747_amd import lyaf as L
    from synth import fields

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    L.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, n):
        """Average seconds of fn() over n calls after one warm-up (HIP events
        on the current stream, which every library call here uses)."""
        fn()
        ev0.record(stream)
        for _ in range(n):
            fn()
        ev1.record(stream)
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / n * 1e-3

    if args.calibrate_copy:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        src = torch.ones(1 << 28, device=dev, dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_per_launch": 2 * src.numel() * 4}))
        return
    if args.fields_only:
        print(json.dumps({"fields_only": True, **fields_section(
            L, torch, dev, fields, timed, max(args.steps, 1))}), flush=True)
        return
    if args.power3d_only:
        print(json.dumps({"power3d_only": True, **power3d_section(
            L, torch, dev, fields, timed, max(args.steps, 1))}), flush=True)
        return
    if args.adjoint_only or args.instrument_only or args.stats_only:
        if args.adjoint_only:
            print(json.dumps({"adjoint_only": True, **adjoint_section(
                L, torch, dev, fields, timed, max(args.steps, 1), None)}), flush=True)
            return
        w = fields.config2()
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        d = [t(x) for x in (w.delta, w.vpec, w.dv, w.T0, w.gamma)]
        raw = torch.empty(w.n_pix, device=dev, dtype=torch.float32)
        F = torch.empty_like(raw)
        A = torch.empty((), device=dev, dtype=torch.float64)
        L.tau(*d, w.offsets, raw, window_k=w.window_k)
        L.normalise_mean_flux(raw, F, w.target_F, A)
        if args.stats_only:
            print(json.dumps({"stats_only": True, **stats_section(
                L, torch, dev, timed, max(args.steps, 1), F, d[2], w)}), flush=True)
            return
        print(json.dumps({"instrument_only": True, **instrument_section(
            L, torch, dev, fields, timed, max(args.steps, 1), F, d[2], w)}), flush=True)
        return
    peak = None
    if not args.no_peaks and not args.tau_only:
        from paper_1105_4747_amd import peaks as PK
        peak = PK.measure()
        print(f"bench: peaks {json.dumps(peak)}", file=sys.stderr, flush=True)
    w = getattr(fields, args.workload)()
    print(f"bench: workload {w.name}, P={w.n_pix}", file=sys.stderr, flush=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    delta, vpec, dvt, T0, gamma = t(w.delta), t(w.vpec), t(w.dv), t(w.T0), t(w.gamma)
    P = w.n_pix
    ts = torch.empty(P, device=dev, dtype=torch.float32)
    F = torch.empty(P, device=dev, dtype=torch.float32)
    A = torch.empty((), device=dev, dtype=torch.float64)

    if args.tau_only:
        shape = 4 if args.shape is None else args.shape
        fl = L.FLAG_SHAPE(shape) | (L.FLAG_PERSISTENT if args.persistent else 0)
        for _ in range(args.warmup + args.steps):
            L.tau(delta, vpec, dvt, T0, gamma, w.offsets, ts, tau_ref=w.tau_ref,
                  delta_pivot=w.delta_pivot, window_k=w.window_k, flags=fl)
        torch.cuda.synchronize()
        print(json.dumps({"tau_only": True, "shape": shape, "persistent": args.persistent,
                          "launches": args.warmup + args.steps}), flush=True)
        return

    # the whole forward (reach, windowed tau, mean-flux root-find, tau', F) as
    # one tuned plan, replayed from a hipGraph
    plan = L.Plan(delta, vpec, dvt, T0, gamma, w.offsets, w.target_F, ts, F, A,
                  tau_ref=w.tau_ref, delta_pivot=w.delta_pivot, window_k=w.window_k,
                  autotune=True)
    info = plan.describe()
    print(f"bench: plan {json.dumps(info)}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        plan.execute()
    torch.cuda.synchronize()
    if plan.status() != 0:
        raise RuntimeError("device status set during warmup")

    # timed region: exactly K steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.execute()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = P * args.steps / elapsed
    print(f"bench: {ms_per_step:.4f} ms/step, {value:.4e} px/s", file=sys.stderr, flush=True)

    # the windowed tau kernel alone (the plan's shape and launch form): HIP
    # events recorded by the library around that launch, on its stream
    shape = info["shape"]
    pers = info["persistent_grid"] > 0
    tau_flags = L.FLAG_SHAPE(shape) | (L.FLAG_PERSISTENT if pers else 0)
    raw = torch.empty(P, device=dev, dtype=torch.float32)

    def tau_stage(out, flags=tau_flags):
        L.tau(delta, vpec, dvt, T0, gamma, w.offsets, out, tau_ref=w.tau_ref,
              delta_pivot=w.delta_pivot, window_k=w.window_k, flags=flags)

    reps = max(args.steps, 10)
    t_kernel = kernel_seconds(L, lambda: tau_stage(raw), reps, "tau")
    t_reach = kernel_seconds(L, lambda: tau_stage(raw), reps, "reach")
    t_tau = timed(lambda: tau_stage(raw), reps)
    tmp = torch.empty_like(raw)
    t_norm = kernel_seconds(L, lambda: (tmp.copy_(raw), L.normalise_mean_flux(tmp, F, w.target_F,
                                                                            A)),
                            reps, "normalise")
    t_eager = timed(lambda: (tau_stage(raw, 0), L.normalise_mean_flux(tmp.copy_(raw), F,
                                                                       w.target_F, A)), reps)
    tau_stage(raw)  # raw tau of this workload for the error check
    pairs = algorithmic_pairs(w)
    roofline = tau_roofline(pairs, t_kernel, tau_kernel_name(shape, pers), peak)
    roofline["traffic"] = measured_traffic(shape, pers, w.name)
    roofline["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE)"
    roofline["pairs_per_px"] = round(pairs / P, 3)
    extra = {"plan": info, "tau_kernel_ms": round(t_kernel * 1e3, 4),
             "reach_kernel_ms": round(t_reach * 1e3, 4),
             "tau_stage_ms": round(t_tau * 1e3, 4),
             "normalise_stage_ms": round(t_norm * 1e3, 4),
             "eager_step_ms": round(t_eager * 1e3, 4)}

    if not args.no_plain:
        # the plain unbatched FP32 kernel (full O(N^2) sum, one launch per skewer)
        plain = torch.empty_like(raw)
        t_plain = timed(lambda: tau_stage(plain, L.FLAG_PLAIN), 1)
        extra["plain_fp32_tau_px_per_s"] = P / t_plain
        extra["plain_fp32_tau_ms"] = round(t_plain * 1e3, 3)
        extra["speedup_tau_vs_plain"] = round(t_plain / t_tau, 2)
        del plain

    if not args.no_batched:
        extra["batched"] = batched_section(L, torch, dev, fields, timed, reps, peak)
    if not args.no_box:
        extra["box"] = box_section(L, torch, dev, fields, timed, 5, peak)
    if not args.no_adjoint:
        extra["adjoint"] = adjoint_section(L, torch, dev, fields, timed, reps, peak)
    if not args.no_instrument:
        plan.execute()  # F of this workload
        extra["instrument"] = instrument_section(L, torch, dev, fields, timed, reps, F, dvt, w)
    if not args.no_fields:
        extra["field_synthesis"] = fields_section(L, torch, dev, fields, timed, reps)
        torch.cuda.empty_cache()
    if not args.no_power3d:
        extra["flux_power_3d"] = power3d_section(L, torch, dev, fields, timed, reps)
        torch.cuda.empty_cache()
    if not args.no_stats:
        plan.execute()  # F of this workload
        extra["flux_stats"] = stats_section(L, torch, dev, timed, reps, F, dvt, w)
    if peak is not None:
        extra["peaks"] = {k: peak[k] for k in ("fma_lane_ops_per_s", "trans_lane_ops_per_s",
                                               "mix_fma_per_exp", "mix_exp_per_s",
                                               "pair_per_s_exp", "pair_per_s_noexp",
                                               "pair_peak_per_s", "copy_bytes_per_s")}
    plan.close()

    cpu = error = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu, sub, raw_ref, F_ref = cpu_baseline(w)
        error = error_vs_oracle(L, torch, dev, raw, sub, raw_ref, F_ref)

    out = {
        "metric": METRIC, "value": value, "unit": "skewer-pixels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_skewers": w.n_skewers, "n_pix": P,
                   "dv_kms": float(w.dv[0]), "T0": float(w.T0[0]), "gamma": float(w.gamma[0]),
                   "window_k": w.window_k, "target_F": w.target_F,
                   "parallelism": "single GPU"},
        "roofline": roofline, "error": error, "cpu_baseline": cpu, "detail": extra,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
