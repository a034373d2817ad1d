"""Error paths of the C ABI on the GPU: a non-finite
input is reported as HS_ERR_NONFINITE (also a single NaN among many finite
values: every maximum the library checks propagates NaN), an empty sampled
set and a rank-zero fit as HS_ERR_RANK, Newton's iteration limit as
HS_ERR_NOT_CONVERGED; after each the context keeps working (the next call
matches the oracle)."""
import numpy as np
import pytest

import workloads as W
from oracle import fv, hybrid, pod, sampling

from gpu_common import case, ctx_for, dev, host, need_gpu, print_case, rel, torch

pytestmark = pytest.mark.gpu


def setup(name="burgers2d"):
    wl, prob, q0 = case(name, 0)
    snaps = [q0]
    for _ in range(12):
        snaps.append(fv.hdm_step(prob, snaps[-1])[0])
    b = pod.pod(snaps, 12, 8)
    eps, _ = sampling.indicator_full(prob, snaps[-1], b["Phi"], b["psi_new"])
    sel = sampling.select(prob, eps, sampling.RULE_FRACTION, wl.frac)
    return wl, prob, snaps, b, sel


def still_works(ctx, prob, g):
    out, _ = ctx.hdm_step(dev(g))
    qo, _ = fv.hdm_step(prob, g)
    assert rel(host(out), qo) < 1e-12


@pytest.mark.parametrize("name", ["burgers1d", "burgers2d", "euler2d"])
def test_nan_input_is_nonfinite(name):
    need_gpu()
    print_case("error: NaN input", name)
    import paper_2301_01718_amd as hs
    wl, prob, q0 = case(name, 0)
    ctx = ctx_for(prob)
    bad = q0.copy()
    bad[bad.size // 3] = np.nan
    with pytest.raises(hs.HsError) as e:
        ctx.hdm_step(dev(bad))
    assert e.value.status == -5, e.value
    still_works(ctx, prob, q0)


def test_nan_in_hybrid_step_is_nonfinite():
    need_gpu()
    print_case("error: NaN input to the hybrid step")
    import paper_2301_01718_amd as hs
    wl, prob, snaps, b, sel = setup()
    ctx = ctx_for(prob)
    s = ctx.samples_set(dev(sel["hat"]))
    Phi = dev(np.ascontiguousarray(b["Phi"].T).reshape(-1))
    bad = snaps[-1].copy()
    bad[7] = np.inf
    with pytest.raises(hs.HsError) as e:
        ctx.rom_hybrid_step(dev(bad), Phi, dev(b["psi_new"]), b["m_eff"], s)
    assert e.value.status == -5, e.value
    out, info = ctx.rom_hybrid_step(dev(snaps[-1]), Phi, dev(b["psi_new"]), b["m_eff"], s)
    ref = hybrid.hybrid_step(prob, snaps[-1], b["Phi"], b["psi_new"], sel["hat"], sel["tilde"])
    assert rel(host(out), ref["gamma"]) < 1e-12


def test_empty_set_and_rank_zero_fit_are_rank_errors():
    need_gpu()
    print_case("error: empty set, rank-zero fit")
    import paper_2301_01718_amd as hs
    wl, prob, snaps, b, sel = setup()
    ctx = ctx_for(prob)
    Phi_o = b["Phi"]
    psi = dev(b["psi_new"])
    empty = ctx.samples_set(torch.zeros(0, dtype=torch.int32, device="cuda"))
    with pytest.raises(hs.HsError) as e:
        ctx.rom_hybrid_step(dev(snaps[-1]), dev(np.ascontiguousarray(Phi_o.T).reshape(-1)), psi, b["m_eff"], empty)
    assert e.value.status == -4, e.value
    # a basis that vanishes on every sampled row: the fit has rank zero
    Z = Phi_o.copy()
    Z[sel["hat"], :] = 0.0
    s = ctx.samples_set(dev(sel["hat"]))
    with pytest.raises(hs.HsError) as e:
        ctx.rom_hybrid_step(dev(snaps[-1]), dev(np.ascontiguousarray(Z.T).reshape(-1)), psi, b["m_eff"], s)
    assert e.value.status == -4, e.value
    still_works(ctx, prob, snaps[-1])


def test_newton_iteration_limit_is_not_converged():
    need_gpu()
    print_case("error: Newton iteration limit")
    import paper_2301_01718_amd as hs
    wl, prob, q0 = case("burgers2d", 0)
    q1, its = fv.hdm_step(prob, q0)
    assert its >= 2
    ctx = ctx_for(prob, newton_maxit=1)
    with pytest.raises(hs.HsError) as e:
        ctx.hdm_step(dev(q0))
    assert e.value.status == -3, e.value
    # a state one Newton iteration from convergence is still solved
    ctx2 = ctx_for(prob)
    out, info = ctx2.hdm_step(dev(q0))
    assert rel(host(out), q1) < 1e-12
