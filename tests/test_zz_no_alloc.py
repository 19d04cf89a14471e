"""The allocation-free network gradient (tdg_mlp_backward_noalloc) against the
entry point it varies (tdg_mlp_backward with a caller-allocated scratch):
same kernels, same summation order, so the results must be bit-identical.
Two calls in a row, the second with fewer samples (the fixed scratch keeps the
first call's rows beyond the second's, which must not leak into it), and the
documented size limit."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inputs(n, seed, dev):
    import torch

    from paper_1907_02367_amd import tdg

    g = torch.Generator().manual_seed(seed)
    P = tdg.mlp_nparam()
    w32 = 0.3 * torch.randn(P, generator=g)
    wb = torch.empty(P, dtype=torch.int16, device=dev)
    tdg.mlp_round(w32.to(dev), wb)
    x = torch.randn(n, 8, generator=g).to(dev)
    t = torch.randn(n, 7, generator=g).to(dev)
    m = (torch.rand(n, 7, generator=g) < 0.8).float().to(dev)
    return wb, x, t, m


def test_noalloc_gradient_matches_allocating_entry_point():
    import torch

    from paper_1907_02367_amd import tdg

    dev = torch.device("cuda", 0)
    P = tdg.mlp_nparam()
    for n, seed in ((8192, 1), (1000, 2), (37, 3)):
        say(f"[gpu no-alloc] network gradient, n = {n}")
        wb, x, t, m = _inputs(n, seed, dev)
        ref, _ = tdg.mlp_backward(wb, x, t, m, norm=float(n))
        got = torch.full((P + 1,), float("nan"), dtype=torch.float32, device=dev)
        tdg.mlp_backward_noalloc(wb, x, t, m, float(n), got)
        torch.cuda.synchronize()
        a, b = got.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), np.abs(a - b).max()
    # beyond the fixed scratch: a clear error, nothing launched
    wb, x, t, m = _inputs(8193, 4, dev)
    grad = torch.zeros(P + 1, dtype=torch.float32, device=dev)
    with pytest.raises(tdg.TdgError) as ei:
        tdg.mlp_backward_noalloc(wb, x, t, m, 1.0, grad)
    assert ei.value.name == "TDG_EINVAL" and "8192" in str(ei.value)
    torch.cuda.synchronize()
    assert (grad.cpu().numpy() == 0).all()
