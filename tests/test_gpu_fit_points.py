"""The first-order hybrid step with ODEIM points (eq. odeim) as the fit's
rows (eq. red_coord, rom_hybrid_step_fit) and their cells added to the
sampled set (hat-S = G u P), against the oracle on the same inputs; 1D/2D
Burgers and 2D Euler."""
import numpy as np
import pytest

from oracle import hybrid, odeim, pod, sampling

from gpu_common import CASES, case, ctx_for, dev, host, indicator_close, need_gpu, print_case, rel, state_tol
from test_gpu_kernels import window

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", list(CASES))
def test_hybrid_step_with_odeim_fit_matches_oracle(name):
    need_gpu()
    print_case("rom_hybrid_step_fit (ODEIM)", name)
    wl, prob, q0 = case(name, 0)
    w, m = 12, 6
    snaps = window(prob, q0, w)
    o = pod.pod(snaps, w, m)
    Phi_o, psi, me = o["Phi"], o["psi_new"], o["m_eff"]
    g = snaps[-1]
    eps, _ = sampling.indicator_full(prob, g, Phi_o, psi)
    sel = sampling.select(prob, eps, sampling.RULE_FRACTION, wl.frac)
    ctx = ctx_for(prob)
    Phi = dev(np.ascontiguousarray(Phi_o.T).reshape(-1))
    pts = ctx.odeim(Phi, me, 2 * me)
    p_host = host(pts)
    assert p_host.tolist() == odeim.odeim(Phi_o, 2 * me)
    s = ctx.sample_select(dev(eps), wl.frac, halo=wl.halo)
    ctx.samples_add_points(s, pts)
    hat, tilde, _ = (host(t) for t in s.export())
    o_hat = np.union1d(sel["hat"], odeim.cells_of(p_host, prob.ncell)).astype(np.int32)
    assert np.array_equal(hat, o_hat)
    o_tilde = np.flatnonzero(sampling.neighbours(prob, np.isin(np.arange(prob.ncell), o_hat)))
    assert np.array_equal(tilde, o_tilde)
    ref = hybrid.hybrid_step(prob, g, Phi_o, psi, o_hat, o_tilde, fit_points=p_host)
    eps_g, y_g = ctx.empty(prob.ncell), ctx.empty(me)
    out, info = ctx.rom_hybrid_step(dev(g), Phi, dev(psi), me, s, eps=eps_g, y=y_g, fit_points=pts)
    d = rel(host(out), ref["gamma"])
    print(f"  n_s {hat.size} n_p {2 * me} J {info['subiters']}/{ref['J']} y {rel(host(y_g), ref['y']):.3e} "
          f"state {d:.3e} fit_cond {info['fit_cond']:.2e}", flush=True)
    assert info["subiters"] == ref["J"]
    assert d < state_tol(info["fit_cond"], tol=1e-12)
    ok, dd = indicator_close(host(eps_g), ref["eps"], ref["gamma"], tol=1e-12, cell_tol=1e-10)
    assert ok, dd


def test_fit_points_outside_the_state_add_no_row():
    """Fit points outside [0, N) (a caller's list with stale or padded
    entries) add no row to the fit: the step equals the one over the valid
    points alone (the same J; the state to 1e-13, the partial sums only
    regrouped)."""
    need_gpu()
    print_case("rom_hybrid_step_fit (points outside the state)", "burgers2d")
    import torch
    wl, prob, q0 = case("burgers2d", 0)
    w, m = 12, 6
    snaps = window(prob, q0, w)
    o = pod.pod(snaps, w, m)
    Phi_o, psi, me = o["Phi"], o["psi_new"], o["m_eff"]
    g = snaps[-1]
    eps, _ = sampling.indicator_full(prob, g, Phi_o, psi)
    ctx = ctx_for(prob)
    Phi = dev(np.ascontiguousarray(Phi_o.T).reshape(-1))
    pts = ctx.odeim(Phi, me, 2 * me)
    s = ctx.sample_select(dev(eps), wl.frac, halo=wl.halo)
    ctx.samples_add_points(s, pts)
    padded = torch.cat([pts, torch.tensor([-1, prob.n, prob.n + 7, -(2 ** 31)], dtype=torch.int32,
                                          device=pts.device)])
    out1, info1 = ctx.rom_hybrid_step(dev(g), Phi, dev(psi), me, s, fit_points=pts)
    ref = host(out1).copy()
    out2, info2 = ctx.rom_hybrid_step(dev(g), Phi, dev(psi), me, s, fit_points=padded)
    d = rel(host(out2), ref)
    print(f"  J {info2['subiters']}/{info1['subiters']} state {d:.3e}", flush=True)
    assert info2["subiters"] == info1["subiters"]
    assert d < 1e-13
