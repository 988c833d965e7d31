"""Helpers shared by the GPU parity tests: upload a workload, run the library
through its C ABI (via the ctypes binding), and the tolerances of the parity
bar.  Tolerances:
  tau   |tau_gpu - tau_ref| <= 1e-5 * max(tau_ref, 1e-3)
  F     |F_gpu - F_ref| <= 1e-6
  A     |A_gpu / A_ref - 1| <= 1e-7 (A_ref: the oracle root-find on the GPU's raw tau)
  grads ||g_gpu - g_ref||_inf <= 1e-4 ||g_ref||_inf per array; T0 and gamma
        gradients relative 1e-4 (per skewer, against the largest magnitude)
"""
import numpy as np

TAU_REL, TAU_FLOOR, F_ABS, A_REL, G_REL = 1e-5, 1e-3, 1e-6, 1e-7, 1e-4


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


def assert_grad_close(gpu, ref, what, rel=G_REL):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max()
    err = np.abs(gpu - ref).max()
    assert err <= rel * scale, f"{what}: max err {err:.3g} vs scale {scale:.3g}"
    return err / scale if scale else 0.0


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


def assert_subset_flux(raw_gpu_sub, ref_sub, target_F, what="subset F"):
    """F parity on a subset normalised on its own on both sides: the GPU
    rescales its own raw tau of the subset, the oracle its own (no value
    crosses from one side to the other)."""
    from oracle import oracle as O
    _, F_gpu, _ = gpu_normalise(to_dev(np.ascontiguousarray(raw_gpu_sub, np.float32)), target_F)
    _, F_ref, _ = O.normalise(np.asarray(ref_sub, np.float64), target_F)
    return assert_F_close(F_gpu.cpu().numpy(), F_ref, what)
