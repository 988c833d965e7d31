"""Helpers shared by the GPU parity tests: upload a workload, run the library
through its C ABI (via the ctypes binding), and the tolerances of the parity
bar.  Tolerances:
  tau   |tau_gpu - tau_ref| <= 1e-5 * max(tau_ref, 1e-3)
  F     |F_gpu - F_ref| <= 1e-6
  A     |A_gpu / A_ref - 1| <= 1e-7 (A_ref: the oracle root-find on the GPU's raw tau)
  grads ||g_gpu - g_ref||_inf <= 1e-4 ||g_ref||_inf per array, and per element
        |g_gpu - g_ref| <= 1e-3 |g_ref| wherever |g_ref| > 1e-2 ||g_ref||_inf;
        the per-skewer T0 and gamma gradients each within 1e-4 of their own
        reference value
"""
import numpy as np

TAU_REL, TAU_FLOOR, F_ABS, A_REL, G_REL = 1e-5, 1e-3, 1e-6, 1e-7, 1e-4
G_ELEM_REL, G_ELEM_FLOOR, G_SKEWER_REL = 1e-3, 1e-2, 1e-4


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    if isinstance(a, torch.Tensor):
        return a.to(dev()).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


class OnDevice:
    """A workload's arrays on the GPU."""

    def __init__(self, w):
        self.w = w
        self.delta, self.vpec = to_dev(w.delta), to_dev(w.vpec)
        self.dv, self.T0, self.gamma = to_dev(w.dv), to_dev(w.T0), to_dev(w.gamma)
        self.offsets = np.asarray(w.offsets, np.int64)


def gpu_tau(w, flags=0, window_k=None, d=None, tau_ref=None, delta_pivot=None):
    import torch
    from paper_1105_4747_amd import lyaf as L
    d = d or OnDevice(w)
    out = torch.full((w.n_pix,), float("nan"), device=dev(), dtype=torch.float32)
    L.tau(d.delta, d.vpec, d.dv, d.T0, d.gamma, d.offsets, out,
          tau_ref=w.tau_ref if tau_ref is None else tau_ref,
          delta_pivot=w.delta_pivot if delta_pivot is None else delta_pivot,
          window_k=w.window_k if window_k is None else window_k, flags=flags)
    torch.cuda.synchronize()
    return out


def gpu_normalise(raw, target_F):
    import torch
    from paper_1105_4747_amd import lyaf as L
    ts = raw.clone()
    F = torch.empty_like(raw)
    A = torch.empty((), device=raw.device, dtype=torch.float64)
    L.normalise_mean_flux(ts, F, target_F, A)
    torch.cuda.synchronize()
    return ts, F, A


def assert_tau_close(gpu, ref, what="tau"):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    assert gpu.shape == ref.shape
    assert np.all(np.isfinite(gpu)), f"{what}: non-finite values"
    err = np.abs(gpu - ref)
    tol = TAU_REL * np.maximum(ref, TAU_FLOOR)
    bad = err > tol
    worst = float(np.max(err / tol)) if err.size else 0.0
    assert not bad.any(), (f"{what}: {bad.sum()} of {bad.size} outside tolerance; "
                           f"worst err/tol {worst:.3g} at {int(np.argmax(err / tol))}")
    return worst


def assert_F_close(gpu, ref, what="F"):
    err = np.abs(np.asarray(gpu, np.float64) - np.asarray(ref, np.float64))
    assert float(err.max()) <= F_ABS, f"{what}: max |dF| {err.max():.3g}"
    return float(err.max())


def assert_grad_close(gpu, ref, what, rel=G_REL, elem_rel=G_ELEM_REL):
    """Max-norm bar per array, then the per-element relative bar on every
    element whose reference is above 1e-2 of the largest.  Returns the max-norm
    ratio and prints both."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    assert gpu.shape == ref.shape and np.all(np.isfinite(gpu)), f"{what}: shape or non-finite"
    scale = np.abs(ref).max() if ref.size else 0.0
    err = np.abs(gpu - ref).max() if ref.size else 0.0
    assert err <= rel * scale, f"{what}: max err {err:.3g} vs scale {scale:.3g}"
    big = np.abs(ref) > G_ELEM_FLOOR * scale
    worst = 0.0
    if big.any():
        r = np.abs(gpu[big] - ref[big]) / np.abs(ref[big])
        worst = float(r.max())
        assert worst <= elem_rel, (f"{what}: {int((r > elem_rel).sum())} of {int(big.sum())} "
                                   f"large elements off by more than {elem_rel:g} relative "
                                   f"(worst {worst:.3g})")
    print(f"{what}: max-norm {err / scale if scale else 0.0:.2e}, "
          f"worst large-element relative {worst:.2e}")
    return err / scale if scale else 0.0


def assert_per_skewer_close(gpu, ref, what, rel=G_SKEWER_REL):
    """Per-skewer scalar gradients (dL/dT0, dL/dgamma): each within ``rel`` of
    its own reference value."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    assert gpu.shape == ref.shape and np.all(np.isfinite(gpu)), f"{what}: shape or non-finite"
    r = np.abs(gpu - ref) / np.abs(ref)
    worst = float(r.max()) if r.size else 0.0
    assert np.all(np.abs(gpu - ref) <= rel * np.abs(ref)), (
        f"{what}: {int((r > rel).sum())} of {r.size} skewers off by more than {rel:g} "
        f"relative (worst {worst:.3g} at skewer {int(np.argmax(r))})")
    print(f"{what}: worst per-skewer relative {worst:.2e}")
    return worst


def assert_mean_flux_root(tau, A, target_F, what="A", rel=A_REL):
    """The mean-flux condition holds for the GPU's own outputs (a property that
    holds at any size; no oracle): g(A) = <exp(-A tau)> - target_F must be zero
    to within the A bar, |g| <= rel * A * |g'(A)|, g' = -<tau exp(-A tau)>."""
    t = np.asarray(tau, np.float64)
    e = np.exp(-A * t)
    g = float(e.mean()) - target_F
    dg = float((t * e).mean())
    assert abs(g) <= rel * A * dg, f"{what}: g(A) = {g:.3g}, allowed {rel * A * dg:.3g}"
    return abs(g) / (A * dg)


def mean_flux_residual_chunked(raw_dev, A, target_F, chunk=1 << 26):
    """g(A) = <exp(-A tau)> - target_F and g'(A) = -<tau exp(-A tau)> over every
    value of a device tensor, copied to the host chunk by chunk and summed in
    FP64 (for arrays too large to copy at once)."""
    import math
    n = int(raw_dev.numel())
    s0, s1 = [], []
    for a in range(0, n, chunk):
        t = raw_dev[a:a + chunk].cpu().numpy().astype(np.float64)
        e = np.exp(-A * t)
        s0.append(float(e.sum()))
        s1.append(float((t * e).sum()))
    return math.fsum(s0) / n - target_F, math.fsum(s1) / n


def assert_subset_flux(raw_gpu_sub, ref_sub, target_F, what="subset F"):
    """F parity on a subset normalised on its own on both sides: the GPU
    rescales its own raw tau of the subset, the oracle its own (no value
    crosses from one side to the other)."""
    from oracle import oracle as O
    _, F_gpu, _ = gpu_normalise(to_dev(np.ascontiguousarray(raw_gpu_sub, np.float32)), target_F)
    _, F_ref, _ = O.normalise(np.asarray(ref_sub, np.float64), target_F)
    return assert_F_close(F_gpu.cpu().numpy(), F_ref, what)
