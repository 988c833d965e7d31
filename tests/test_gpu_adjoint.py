"""GPU parity of the hand-written adjoint (lyaf_tau_backward and
lyaf_normalise_mean_flux_backward, also through the autograd wrapper) against
the oracle's chain-rule gradient, and against central finite differences of
the FP64 oracle forward."""
import numpy as np
import pytest

from gpu_util import (OnDevice, assert_grad_close, assert_per_skewer_close, gpu_normalise,
                      gpu_tau, to_dev)
from oracle import oracle as O
from synth import fields

pytestmark = pytest.mark.gpu


def _oracle_F(w, T0=None, gamma=None):
    raw = O.tau(w.delta, w.vpec, w.dv, w.T0 if T0 is None else T0,
                w.gamma if gamma is None else gamma, offsets=w.offsets)
    return O.normalise(raw, w.target_F)


def test_tau_backward_random_cotangent():
    import torch
    from paper_1105_4747_amd import lyaf as L
    w = fields.config1().subset(range(6))
    d = OnDevice(w)
    rng = np.random.default_rng(1)
    g = rng.normal(size=w.n_pix).astype(np.float32)
    gd = torch.empty_like(d.delta)
    gv = torch.empty_like(d.vpec)
    gT = torch.empty(w.n_skewers, device="cuda:0", dtype=torch.float64)
    gg = torch.empty_like(gT)
    print(f"case: adjoint {w.name} random cotangent", flush=True)
    L.tau_backward(d.delta, d.vpec, d.dv, d.T0, d.gamma, d.offsets, to_dev(g), gd, gv, gT, gg,
                   window_k=w.window_k)
    torch.cuda.synchronize()
    rd, rv, rT, rg = O.tau_grad(w.delta, w.vpec, w.dv, w.T0, w.gamma, g.astype(np.float64),
                                offsets=w.offsets)
    assert_grad_close(gd.cpu().numpy(), rd, "dL/dDelta")
    assert_grad_close(gv.cpu().numpy(), rv, "dL/dv")
    assert_per_skewer_close(gT.cpu().numpy(), rT, "dL/dT0")
    assert_per_skewer_close(gg.cpu().numpy(), rg, "dL/dgamma")


@pytest.mark.parametrize("n_pix,dv", [(256, 2.0), (40, 3.0)])
def test_tau_backward_full_box_path(n_pix, dv):
    import torch
    from paper_1105_4747_amd import lyaf as L
    w = fields.small_workload(n_skewers=3, n_pix=n_pix, seed=9, dv=dv)
    d = OnDevice(w)
    g = np.random.default_rng(2).normal(size=w.n_pix).astype(np.float32)
    gd, gv = torch.empty_like(d.delta), torch.empty_like(d.vpec)
    gT = torch.empty(3, device="cuda:0", dtype=torch.float64)
    gg = torch.empty_like(gT)
    L.tau_backward(d.delta, d.vpec, d.dv, d.T0, d.gamma, d.offsets, to_dev(g), gd, gv, gT, gg)
    torch.cuda.synchronize()
    rd, rv, rT, rg = O.tau_grad(w.delta, w.vpec, w.dv, w.T0, w.gamma, g.astype(np.float64),
                                offsets=w.offsets)
    assert_grad_close(gd.cpu().numpy(), rd, "dL/dDelta")
    assert_grad_close(gv.cpu().numpy(), rv, "dL/dv")
    assert_per_skewer_close(gT.cpu().numpy(), rT, "dL/dT0")
    assert_per_skewer_close(gg.cpu().numpy(), rg, "dL/dgamma")


def test_normalise_backward_against_oracle():
    import torch
    from paper_1105_4747_amd import lyaf as L
    w = fields.config1()
    # both sides take the oracle's raw tau, rounded to float32, as input
    raw32 = O.tau(w.delta, w.vpec, w.dv, w.T0, w.gamma, offsets=w.offsets).astype(np.float32)
    raw = to_dev(raw32)
    ts, F, A = gpu_normalise(raw, w.target_F)
    rng = np.random.default_rng(3)
    gF = rng.normal(size=w.n_pix).astype(np.float32)
    gT = rng.normal(size=w.n_pix).astype(np.float32)
    raw64 = raw32.astype(np.float64)
    A_ref, _ = O.mean_flux_A(raw64, w.target_F)
    for implicit in (True, False):
        out = torch.empty_like(raw)
        L.normalise_mean_flux_backward(raw, A, to_dev(gF), to_dev(gT), implicit, out)
        torch.cuda.synchronize()
        ref = O.normalise_backward(raw64, A_ref, grad_F=gF.astype(np.float64),
                                   grad_tau_scaled=gT.astype(np.float64), implicit_A=implicit)
        assert_grad_close(out.cpu().numpy(), ref, f"dL/dtau implicit={implicit}", rel=1e-5)


def _c5_subset(n=16):
    w = fields.config5().subset(range(n))
    _, F_t, _ = _oracle_F(w, T0=1.1 * w.T0.astype(np.float64),
                          gamma=w.gamma.astype(np.float64) + 0.05)
    return w, F_t


def test_autograd_config5_subset_against_oracle_and_fd():
    """Config 5's loss L = sum (F - F_t)^2, F_t from (1.1 T0, gamma + 0.05), on a
    16-skewer subset normalised on its own (both sides).  Gradient through
    TauFlux vs the oracle's chain rule; the oracle's chain rule vs central FD of
    the oracle forward along random directions."""
    import torch
    from paper_1105_4747_amd import lyaf as L
    w, F_t = _c5_subset()
    d = OnDevice(w)
    delta = d.delta.clone().requires_grad_(True)
    vpec = d.vpec.clone().requires_grad_(True)
    T0 = d.T0.clone().requires_grad_(True)
    gamma = d.gamma.clone().requires_grad_(True)
    print(f"case: {w.name} autograd", flush=True)
    ts, F, A = L.tau_flux(delta, vpec, T0, gamma, d.dv, w.offsets, w.target_F,
                          window_k=w.window_k)
    loss = ((F.double() - to_dev(F_t)) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    raw = O.tau(w.delta, w.vpec, w.dv, w.T0, w.gamma, offsets=w.offsets)
    _, F_ref, A_ref = O.normalise(raw, w.target_F)
    g_raw = O.normalise_backward(raw, A_ref, grad_F=2 * (F_ref - F_t), implicit_A=True)
    rd, rv, rT, rg = O.tau_grad(w.delta, w.vpec, w.dv, w.T0, w.gamma, g_raw, offsets=w.offsets)
    assert_grad_close(delta.grad.cpu().numpy(), rd, "dL/dDelta")
    assert_grad_close(vpec.grad.cpu().numpy(), rv, "dL/dv")
    assert_per_skewer_close(T0.grad.cpu().numpy(), rT, "dL/dT0")
    assert_per_skewer_close(gamma.grad.cpu().numpy(), rg, "dL/dgamma")

    # central FD of the oracle forward (A re-solved) along random directions
    def Lf(dd, vv, TT, gg):
        r = O.tau(dd, vv, w.dv, TT, gg, offsets=w.offsets)
        _, Fx, _ = O.normalise(r, w.target_F)
        return float(((Fx - F_t) ** 2).sum())

    rng = np.random.default_rng(8)
    d0, v0 = w.delta.astype(np.float64), w.vpec.astype(np.float64)
    T00, g00 = w.T0.astype(np.float64), w.gamma.astype(np.float64)
    gd_gpu = delta.grad.cpu().numpy().astype(np.float64)
    gv_gpu = vpec.grad.cpu().numpy().astype(np.float64)
    for _ in range(2):
        ud = rng.normal(size=w.n_pix) * d0 * (np.abs(d0 - 10) > 1e-3)
        uv = rng.normal(size=w.n_pix)
        h = 1e-6
        fd = (Lf(d0 + h * ud, v0 + h * uv, T00, g00) - Lf(d0 - h * ud, v0 - h * uv, T00, g00)) / (2 * h)
        an = float(gd_gpu @ ud + gv_gpu @ uv)
        assert abs(an - fd) <= 1e-3 * abs(fd) + 1e-9, (an, fd)


@pytest.mark.slow
def test_config5_full_size_sampled():
    """4096 x 2048 forward + backward in the benchmark launch shape.  The oracle
    runs its own chain on the whole batch (tau in its windowed mode with
    k = 8, pinned against the full sum; its own A and F; the implicit-A
    correction couples all skewers), and the adjoint of 8 sampled skewers is
    compared; the loss target F_t is a seeded synthetic flux."""
    import torch
    from paper_1105_4747_amd import lyaf as L
    w = fields.config5()
    d = OnDevice(w)
    print(f"case: {w.name} full-size adjoint", flush=True)
    raw = gpu_tau(w, d=d)
    ts, F, A = gpu_normalise(raw, w.target_F)
    F_t = fields.synthetic_flux(np.diff(w.offsets), 55).astype(np.float64)
    gF = (2 * (F.double() - to_dev(F_t))).float()
    g_raw = torch.empty_like(raw)
    L.normalise_mean_flux_backward(raw, A, gF, None, True, g_raw)
    gd, gv = torch.empty_like(d.delta), torch.empty_like(d.vpec)
    gT = torch.empty(w.n_skewers, device="cuda:0", dtype=torch.float64)
    gg = torch.empty_like(gT)
    L.tau_backward(d.delta, d.vpec, d.dv, d.T0, d.gamma, d.offsets, g_raw, gd, gv, gT, gg)
    torch.cuda.synchronize()
    # the oracle's own chain
    raw_ref = O.tau(w.delta, w.vpec, w.dv, w.T0, w.gamma, offsets=w.offsets, window_k=8.0)
    _, F_ref, A_ref = O.normalise(raw_ref, w.target_F)
    g_ref = O.normalise_backward(raw_ref, A_ref, grad_F=2 * (F_ref - F_t), implicit_A=True)
    assert_grad_close(g_raw.cpu().numpy(), g_ref, "dL/dtau_raw", rel=1e-4)
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(w.n_skewers, 8, replace=False))
    sub = w.subset(pick)
    sel = np.concatenate([np.arange(w.offsets[s], w.offsets[s + 1]) for s in pick])
    rd, rv, rT, rg = O.tau_grad(sub.delta, sub.vpec, sub.dv, sub.T0, sub.gamma, g_ref[sel],
                                offsets=sub.offsets)
    assert_grad_close(gd.cpu().numpy()[sel], rd, "dL/dDelta (sampled)")
    assert_grad_close(gv.cpu().numpy()[sel], rv, "dL/dv (sampled)")
    assert_per_skewer_close(gT.cpu().numpy()[pick], rT, "dL/dT0 (sampled)")
    assert_per_skewer_close(gg.cpu().numpy()[pick], rg, "dL/dgamma (sampled)")
    # the adjoint alone on the same input: both sides take the oracle's
    # dL/dtau_raw of the sampled skewers, rounded to float32
    g32 = np.ascontiguousarray(g_ref[sel], np.float32)
    ds = OnDevice(sub)
    gd2, gv2 = torch.empty_like(ds.delta), torch.empty_like(ds.vpec)
    gT2 = torch.empty(sub.n_skewers, device="cuda:0", dtype=torch.float64)
    gg2 = torch.empty_like(gT2)
    L.tau_backward(ds.delta, ds.vpec, ds.dv, ds.T0, ds.gamma, ds.offsets, to_dev(g32), gd2, gv2,
                   gT2, gg2)
    torch.cuda.synchronize()
    rd2, rv2, rT2, rg2 = O.tau_grad(sub.delta, sub.vpec, sub.dv, sub.T0, sub.gamma,
                                    g32.astype(np.float64), offsets=sub.offsets)
    assert_grad_close(gd2.cpu().numpy(), rd2, "dL/dDelta (same input)")
    assert_grad_close(gv2.cpu().numpy(), rv2, "dL/dv (same input)")
    assert_per_skewer_close(gT2.cpu().numpy(), rT2, "dL/dT0 (same input)")
    assert_per_skewer_close(gg2.cpu().numpy(), rg2, "dL/dgamma (same input)")
    del F_ref
