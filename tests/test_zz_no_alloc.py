"""The allocation-free mean-flux rescale (lyaf_normalise_mean_flux_noalloc)
against the allocating entry point lyaf_normalise_mean_flux: the same kernels
on the same raw tau, so tau', F and A must agree bitwise.  Two calls in a row
(the second on a smaller batch, reusing the shared static scratch), then the
status output on a batch without a root."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _raw_tau(n, seed):
    # positive optical depths with a lognormal spread and a ragged length
    rng = np.random.default_rng(seed)
    return np.exp(rng.normal(-1.0, 1.5, n)).astype(np.float32)


def _both(raw_np, target_F):
    import torch
    from paper_1105_4747_amd import lyaf as L
    dev = torch.device("cuda:0")
    raw = torch.from_numpy(raw_np).to(dev)
    t1, t2 = raw.clone(), raw.clone()
    F1, F2 = torch.full_like(raw, float("nan")), torch.full_like(raw, float("nan"))
    A1 = torch.zeros((), device=dev, dtype=torch.float64)
    A2 = torch.zeros((), device=dev, dtype=torch.float64)
    st = torch.zeros((), device=dev, dtype=torch.int32)
    L.normalise_mean_flux(t1, F1, target_F, A1)
    L.normalise_mean_flux_noalloc(t2, F2, target_F, A2, status=st)
    torch.cuda.synchronize()
    assert L.status_read() == 0
    return (t1.cpu().numpy(), F1.cpu().numpy(), float(A1.cpu()),
            t2.cpu().numpy(), F2.cpu().numpy(), float(A2.cpu()), int(st.cpu()))


@pytest.mark.parametrize("first,second", [(3_000_001, 40_963), (1_048_576, 5)])
def test_noalloc_matches_the_allocating_entry_point(first, second):
    for n, seed in ((first, 1), (second, 2)):
        print(f"noalloc normalise: n_pix={n} seed={seed}", flush=True)
        t1, F1, A1, t2, F2, A2, st = _both(_raw_tau(n, seed), 0.75)
        assert st == 0
        assert A1 == A2 and np.isfinite(A1) and A1 > 0
        assert np.array_equal(t1, t2)
        assert np.array_equal(F1, F2)
        # and the root is the root: <exp(-A tau)> = target (FP64 check on the host)
        raw = _raw_tau(n, seed).astype(np.float64)
        assert abs(np.mean(np.exp(-A2 * raw)) - 0.75) <= 1e-9


def test_noalloc_reports_no_root_through_its_status_word():
    import torch
    from paper_1105_4747_amd import lyaf as L
    dev = torch.device("cuda:0")
    raw = torch.zeros(4097, device=dev, dtype=torch.float32)
    raw[:100] = 1.0  # 97.6 % of the pixels have tau = 0 > target 0.5: no root
    F = torch.empty_like(raw)
    A = torch.zeros((), device=dev, dtype=torch.float64)
    st = torch.zeros((), device=dev, dtype=torch.int32)
    print("noalloc normalise: no-root batch", flush=True)
    L.normalise_mean_flux_noalloc(raw, F, 0.5, A, status=st)
    torch.cuda.synchronize()
    assert int(st.cpu()) & L.STATUS_NOROOT
    assert L.status_read() == 0  # the workspace status word is untouched
