"""The allocation-free indicator entry point (hs_indicator_full_noalloc)
against hs_indicator_full: two calls in a row through the C ABI, the second
on a smaller problem (fewer cells, one component instead of four, fewer
modes), each equal to the context entry point's output to the bit (the same
kernels in the same order), in FP64 and with the FP32 basis."""
import numpy as np
import pytest

import workloads as W

from gpu_common import ctx_for, dev, host, need_gpu, print_case, torch

pytestmark = pytest.mark.gpu


def inputs(name, nx, ny, m, seed):
    wl = W.WORKLOADS[name].resized(nx, ny)
    prob, q0 = W.make(wl, seed)
    rng = np.random.default_rng(seed)
    Phi, _ = np.linalg.qr(rng.standard_normal((prob.n, m)))
    psi = q0 + 1e-3 * rng.standard_normal(prob.n)
    gamma = q0 + 1e-2 * rng.standard_normal(prob.n)
    return prob, gamma, Phi, psi


@pytest.mark.parametrize("fp32", [False, True])
def test_noalloc_indicator_equals_context_entry(fp32):
    need_gpu()
    from paper_2301_01718_amd._lib import indicator_full_noalloc
    for name, nx, ny, m, seed in [("euler2d_512", 67, 53, 40, 1), ("burgers1d_1k", 1000, 1, 7, 2)]:
        print_case("indicator noalloc", name, nx, ny, m, "fp32" if fp32 else "fp64")
        prob, gamma, Phi, psi = inputs(name, nx, ny, m, seed)
        P = dev(np.ascontiguousarray(Phi.T).reshape(-1))
        if fp32:
            P = P.to(torch.float32)
        g, s = dev(gamma), dev(psi)
        ctx = ctx_for(prob)
        e_ref, y_ref = ctx.indicator_full(g, P, s, m)
        eps = torch.full((prob.ncell,), -1.0, dtype=torch.float64, device="cuda")
        y = torch.full((m,), -1.0, dtype=torch.float64, device="cuda")
        indicator_full_noalloc(g, P, s, m, prob.ncell, prob.ncomp, eps, y)
        torch.cuda.synchronize()
        assert torch.equal(eps, e_ref) and torch.equal(y, y_ref[:m]), name
        assert host(eps).max() > 0


def test_noalloc_rejects_sizes_beyond_its_array():
    need_gpu()
    from paper_2301_01718_amd._lib import HsError, indicator_full_noalloc
    prob, gamma, Phi, psi = inputs("burgers1d_1k", 100, 1, 3, 0)
    g = dev(gamma)
    P = torch.zeros(65 * prob.n, dtype=torch.float64, device="cuda")
    eps = torch.zeros(prob.ncell, dtype=torch.float64, device="cuda")
    with pytest.raises(HsError):
        indicator_full_noalloc(g, P, g, 65, prob.ncell, 1, eps)
