"""Trajectory parity of the GPU Algorithm-1 driver with the oracle.

Every step is re-computed by the oracle from the GPU's own inputs (the
previous snapshot, the basis and sampled set the GPU used) and compared to
the GPU output: 1e-12 relative state error per step.  Every sampling
decision is re-taken by the oracle on the GPU's indicator (bit-exact sets),
and every basis is compared with the oracle's POD of the GPU's window
(reference state bit for bit, projector and singular values to rounding).
The step schedule must equal an independent oracle run's, and the final
states of the two independent runs are compared to a looser bound, since
rounding-level differences in the bases feed forward."""
import numpy as np
import pytest

import workloads as W
from oracle import arom, fv, hybrid, pod, sampling

from gpu_common import ctx_for, dev, host, need_gpu, print_case, projector_tol, rel, torch

pytestmark = pytest.mark.gpu


def run_checked(wl, seed, steps=None):
    import paper_2301_01718_amd.driver as D
    prob, q0 = W.make(wl, seed)
    steps = steps or wl.steps
    cfg = D.AromConfig(w=wl.w, m=wl.m, z=wl.z, fraction=wl.frac, halo=wl.halo)
    drv = D.Arom(prob, cfg)
    errs, hyb, resync = [], [], []
    snaps = {0: q0.copy()}
    hp = hybrid.HybridParams()

    def on_step(k, rec, used, out):
        qp = host(used["q_prev"])
        g = host(out)
        snaps[k] = g
        if rec["type"] == "hybrid":
            m = used["m"]
            Phi = host(used["Phi"])[: m * prob.n].reshape(m, prob.n).T
            psi = host(used["psi"])
            hat, tilde, _ = used["samples"].export()
            ref = hybrid.hybrid_step(prob, qp, Phi, psi, host(hat), host(tilde), hp)
            errs.append(rel(g, ref["gamma"]))
            hyb.append((k, rec["J"], ref["J"]))
        else:
            ref, _ = fv.hdm_step(prob, qp)
            errs.append(rel(g, ref))

    def on_update(k, rec, st):
        eps = host(st["eps"])
        if st["samples"] is not None:
            o = sampling.select(prob, eps, sampling.RULE_FRACTION, wl.frac, halo=wl.halo)
            hat, tilde, _ = st["samples"].export()
            assert np.array_equal(host(hat), o["hat"]) and np.array_equal(host(tilde), o["tilde"]), k
        lo = k - wl.w if k >= wl.w else 0
        window = [snaps[j] for j in range(lo, k + 1)]
        b = pod.pod(window, wl.w, wl.m)
        assert np.max(np.abs(host(st["psi"]) - b["psi_new"])) <= 1e-15 * np.max(np.abs(b["psi_new"])), k
        assert st["m_eff"] == b["m_eff"], (k, st["m_eff"], b["m_eff"])
        me = b["m_eff"]
        P = host(st["Phi"])[: me * prob.n].reshape(me, prob.n).T
        X = b["X"]
        d = np.linalg.norm(P @ (P.T @ X) - b["Phi"] @ (b["Phi"].T @ X)) / np.linalg.norm(X)
        assert d <= projector_tol(b["sigma"], me), (k, d, projector_tol(b["sigma"], me))

    qT, recs = drv.run(dev(q0), steps, on_step=on_step, on_update=on_update)
    return prob, q0, host(qT), recs, errs, hyb


def test_burgers1d_1k_trajectory():
    need_gpu()
    print_case("trajectory burgers1d_1k")
    wl = W.WORKLOADS["burgers1d_1k"]
    prob, q0, qT, recs, errs, hyb = run_checked(wl, 0)
    print("  max per-step error", max(errs), "hybrid steps", len(hyb), flush=True)
    assert max(errs) < 1e-12
    assert all(a == b for _, a, b in hyb), [h for h in hyb if h[1] != h[2]][:5]
    ref = arom.run(prob, q0, wl.steps, arom.AromParams(w=wl.w, m=wl.m, z=wl.z, fraction=wl.frac))
    types_o = [r["type"] for r in ref["records"]]
    types_g = [r["type"] for r in recs]
    assert types_o == types_g
    assert sum(t == "full" for t in types_g) == 25
    # Independent runs are compared by accuracy, not state: a rounding-level
    # difference (the GPU builds each basis from the window Gram matrix, the
    # oracle from a direct SVD) can resolve a near-tie in the top-k cut
    # differently, after which the two trajectories are different, equally
    # valid AROM solutions.  Per-step parity above (every step recomputed from
    # the GPU's inputs) is the 1e-12 bar; here both runs must carry the same
    # approximation error against the full-HDM trajectory (Sec. 3.1, e_k).
    qH = q0.copy()
    for _ in range(wl.steps):
        qH, _ = fv.hdm_step(prob, qH)
    e_g = arom.relative_l1_error(qT, qH)
    e_o = arom.relative_l1_error(ref["q"], qH)
    d = arom.relative_l1_error(qT, ref["q"])
    print(f"  e_T gpu {e_g:.3e}  oracle {e_o:.3e}  gpu-vs-oracle {d:.3e}", flush=True)
    assert abs(e_g - e_o) <= 0.5 * e_o and d <= e_o


def test_burgers2d_small_trajectory():
    need_gpu()
    print_case("trajectory burgers2d 48x40")
    wl = W.WORKLOADS["burgers2d_1024"].resized(48, 40, m=10)
    prob, q0, qT, recs, errs, hyb = run_checked(wl, 1, steps=wl.w + 30)
    print("  max per-step error", max(errs), "hybrid steps", len(hyb), flush=True)
    assert max(errs) < 1e-12
    assert all(a == b for _, a, b in hyb)
