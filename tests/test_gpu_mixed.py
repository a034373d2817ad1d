"""Mixed precision (FP32 master copy of the basis, FP64 arithmetic).

* basis_update with an FP32 output writes the FP64 basis rounded once: the
  same reference state, singular values and m_eff bit for bit, and
  Phi32 == fp32(Phi64) exactly.
* rom_hybrid_step / hs_indicator_full on the FP32 copy equal the oracle run
  on that same rounded basis (promoted to FP64 exactly) to the FP64 parity
  bound, and the oracle run on the unrounded FP64 basis to 1e-6 (relative
  state error of the mixed mode against FP64).
* A mixed-mode trajectory against an independent FP64 oracle run: while the
  two take the same decisions (step type, sampled sets, J) the state differs
  by at most 1e-6 relative (the FP32 rounding of the basis, 6e-8 per entry,
  can resolve a near-tie of the top-n_g cut differently after some tens of
  steps, and the runs are then different valid trajectories); the final
  state has the accuracy of the FP64 trajectory against the full HDM.
"""
import numpy as np
import pytest

import workloads as W
from oracle import arom, fv, hybrid, pod, sampling
from oracle import adjoint as A

from gpu_common import CASES, case, ctx_for, dev, host, indicator_close, need_gpu, print_case, rel, torch

pytestmark = pytest.mark.gpu


def window(prob, q0, w, extra=1):
    snaps = [q0]
    for _ in range(w - 1 + extra):
        snaps.append(fv.hdm_step(prob, snaps[-1])[0])
    return snaps


@pytest.mark.parametrize("name", list(CASES))
def test_basis_update_fp32_master_copy(name):
    need_gpu()
    print_case("basis_update mixed", name)
    wl, prob, q0 = case(name, 1)
    w, m = 12, 8
    snaps = [dev(s) for s in window(prob, q0, w)]
    ctx = ctx_for(prob)
    P64 = torch.zeros(m * prob.n, dtype=torch.float64, device="cuda")
    P32 = torch.zeros(m * prob.n, dtype=torch.float32, device="cuda")
    psi64, psi32 = ctx.empty(), ctx.empty()
    s64 = torch.zeros(w, dtype=torch.float64, device="cuda")
    s32 = torch.zeros(w, dtype=torch.float64, device="cuda")
    me64 = ctx.basis_update(snaps, w, m, P64, psi64, s64)
    me32 = ctx.basis_update(snaps, w, m, P32, psi32, s32)
    assert me64 == me32
    assert torch.equal(psi64, psi32) and torch.equal(s64, s32)
    n = me64 * prob.n
    assert torch.equal(P32[:n], P64[:n].to(torch.float32))


def hybrid_inputs(name, seed=0):
    wl, prob, q0 = case(name, seed)
    w, m = 12, 8
    snaps = window(prob, q0, w)
    o = pod.pod(snaps, w, m)
    g = snaps[-1]
    eps, _ = sampling.indicator_full(prob, g, o["Phi"], o["psi_new"])
    sel = sampling.select(prob, eps, sampling.RULE_FRACTION, wl.frac)
    return wl, prob, g, o, sel


@pytest.mark.parametrize("name", list(CASES))
def test_hybrid_step_mixed(name):
    need_gpu()
    print_case("rom_hybrid_step mixed", name)
    wl, prob, g, o, sel = hybrid_inputs(name)
    me, psi = o["m_eff"], o["psi_new"]
    P32 = np.ascontiguousarray(o["Phi"].T).astype(np.float32)        # m x N, rows = columns of Phi
    Phi_r = P32.astype(np.float64).T                                   # the rounded basis, exactly
    ctx = ctx_for(prob)
    s = ctx.samples_set(dev(sel["hat"]))
    eps_g = ctx.empty(prob.ncell)
    y_g = ctx.empty(me)
    out, info = ctx.rom_hybrid_step(dev(g), dev(P32.reshape(-1)), dev(psi), me, s, eps=eps_g, y=y_g)
    ref_r = hybrid.hybrid_step(prob, g, Phi_r, psi, sel["hat"], sel["tilde"])
    ref = hybrid.hybrid_step(prob, g, o["Phi"], psi, sel["hat"], sel["tilde"])
    e_r, e_64 = rel(host(out), ref_r["gamma"]), rel(host(out), ref["gamma"])
    print(f"  vs oracle on the rounded basis {e_r:.2e}, vs the FP64 basis {e_64:.2e}", flush=True)
    assert info["subiters"] == ref_r["J"]
    assert e_r < 1e-12
    assert rel(host(y_g), ref_r["y"]) < 1e-10
    ok, d = indicator_close(host(eps_g), ref_r["eps"], ref_r["gamma"], tol=1e-12)
    assert ok, d
    assert e_64 < 1e-6


@pytest.mark.parametrize("name", list(CASES))
def test_indicator_full_mixed(name):
    need_gpu()
    print_case("indicator_full mixed", name)
    wl, prob, g, o, sel = hybrid_inputs(name, 4)
    me = o["m_eff"]
    P32 = np.ascontiguousarray(o["Phi"].T).astype(np.float32)
    ctx = ctx_for(prob)
    eps, y = ctx.indicator_full(dev(g), dev(P32.reshape(-1)), dev(o["psi_new"]), me)
    eo, yo = sampling.indicator_full(prob, g, P32.astype(np.float64).T, o["psi_new"])
    assert rel(host(y), yo) < 1e-12
    ok, d = indicator_close(host(eps), eo, g)
    assert ok, d


def test_mixed_trajectory_burgers1d():
    need_gpu()
    print_case("trajectory mixed burgers1d_1k")
    import paper_2301_01718_amd as hs
    import paper_2301_01718_amd.driver as D
    wl = W.WORKLOADS["burgers1d_1k"]
    prob, q0 = W.make(wl, 0)
    p = arom.AromParams(w=wl.w, m=wl.m, z=wl.z, fraction=wl.frac)
    qo, tape = A.forward_with_tape(prob, q0, wl.steps, p)          # the FP64 oracle, independently
    cfg = D.AromConfig(w=wl.w, m=wl.m, z=wl.z, fraction=wl.frac, halo=wl.halo, precision=hs.MIXED_FP32)
    drv = D.Arom(prob, cfg)
    assert drv.Phi.dtype == torch.float32
    state = {"agree": True, "compared": 0, "worst": 0.0}

    def on_step(k, rec, used, out):
        st = tape[k - 1]
        same = rec["type"] == st["type"]
        if same and rec["type"] == "hybrid":
            hat, tilde, _ = used["samples"].export()
            same = np.array_equal(host(hat), st["hat"]) and rec["J"] == st["J"]
        state["agree"] = state["agree"] and same
        if state["agree"]:
            e = rel(host(out), st["out"])
            state["worst"] = max(state["worst"], e)
            state["compared"] += 1
            assert e <= 1e-6, (k, e)

    qT, recs = drv.run(dev(q0), wl.steps, on_step=on_step)
    qH = q0.copy()
    for _ in range(wl.steps):
        qH, _ = fv.hdm_step(prob, qH)
    e_mixed = arom.relative_l1_error(host(qT), qH)
    e_o = arom.relative_l1_error(qo, qH)
    d = arom.relative_l1_error(host(qT), qo)
    print(f"  steps with the FP64 oracle's decisions {state['compared']}, max state difference "
          f"{state['worst']:.2e}; e_T mixed {e_mixed:.3e} FP64 oracle {e_o:.3e}, mixed-vs-FP64 {d:.3e}", flush=True)
    assert state["compared"] >= 30
    assert abs(e_mixed - e_o) <= 0.5 * e_o and d <= e_o
