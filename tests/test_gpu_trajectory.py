"""Trajectory parity of the GPU Algorithm-1 driver with the oracle, step by
step with resynchronisation.

The GPU driver runs Alg. 1 on its own.  At every step k the oracle recomputes
that step from the GPU's input to it (gamma_{k-1}, and for the sampling and
basis update after step k the GPU's window of snapshots), so a rounding-level
difference of one step cannot grow over the following ones and every step is
held to the single-step bar:

* step type: the schedule of Alg. 1 (equal on both sides);
* full step: the oracle's Newton root from the GPU's gamma_{k-1}, 1e-12
  relative;
* basis update: the oracle's POD of the GPU's window; sigma to 1e-13
  sigma_0, m_eff equal (or, within 1e-9 relative of the cut tau_pod sigma_0,
  a logged near tie), the span within the Wedin bound of both SVDs;
* sampled sets: the oracle's selection from the oracle's indicator of the
  step (computed from the GPU's gamma_k), bit for bit, or a logged near tie
  (the n_g-th and (n_g+1)-th error norms closer than the indicator's
  resolution);
* hybrid step: the oracle's step from the GPU's gamma_{k-1} and sets, with
  the GPU's basis once it has passed the check above (the trailing POD modes
  are only determined to eps sigma_0 / gap by any correct SVD, so the two
  bases are both correct and differ there); J equal, state 1e-12 relative
  (a gate decided by a residual-norm difference at the rounding level may
  flip a filter flag: such a flip is checked to be a tie and logged), the
  indicator cell by cell.
The same step is also computed by the oracle on its own basis and that
difference is reported.
"""
import numpy as np
import pytest

import workloads as W
from oracle import arom, fv, gauss_newton, hybrid, pod, sampling

from gpu_common import dev, fit_tols, host, indicator_close, need_gpu, print_case, projector_tol, rel

pytestmark = pytest.mark.gpu


class _Tapes:
    """Hands the driver one library tape per hybrid step, so that its filter
    masks can be compared with the oracle's."""

    def __init__(self, ctx):
        self.ctx, self.tapes = ctx, {}

    def tape(self, k):
        self.tapes.pop(k - 2, None)
        if k not in self.tapes:
            self.tapes[k] = self.ctx.tape()
        return self.tapes[k]


def gate_flips(k, masks_gpu, masks_o, norms_o, scale):
    """Cells whose filter flag differs between the GPU and the oracle.  Each
    must be a tie of the gate: its two residual norms equal to 1e-12 of the
    state scale (the inputs of the filter agree to about that)."""
    assert [n for n, _ in masks_gpu] == [n for n, _ in masks_o], (k, "different filter passes")
    tie = 1e-12 * scale
    flips = 0
    for (n, mk), (_, mo), (_, r, rf) in zip(masks_gpu, masks_o, norms_o):
        cells = np.flatnonzero(host(mk).astype(bool) != mo)
        if cells.size:
            gap = np.abs(rf[cells] - r[cells])
            assert np.all(gap <= tie), (k, cells[gap > tie], gap[gap > tie], tie)
            flips += int(cells.size)
    return flips


def run_resync(wl, seed, steps, check_from=1, tol=1e-12, gn=False):
    """gn: the hybrid steps with Gauss-Newton subiterations on both sides."""
    import paper_2301_01718_amd.driver as D
    prob, q0 = W.make(wl, seed)
    n = prob.n
    hp = hybrid.HybridParams()
    cfg = D.AromConfig(w=wl.w, m=wl.m, z=wl.z, fraction=wl.frac, halo=wl.halo, gauss_newton=gn)
    drv = D.Arom(prob, cfg)
    if not gn:
        drv.recorder = _Tapes(drv.ctx)

    def step(qp, Phi, psi, hat, tilde, norms=None):
        if gn:
            return gauss_newton.gn_hybrid_step(prob, qp, Phi, psi, hat, tilde, hp)
        return hybrid.hybrid_step(prob, qp, Phi, psi, hat, tilde, hp, norms=norms)
    st = {"eps_o": None, "basis_used": None, "basis_o": None, "sets_o": None, "worst": 0.0, "worst_own": 0.0,
          "ties": [], "checked": 0, "types": []}

    def on_step(k, rec, used, out):
        st["types"].append(rec["type"])
        if k < check_from:
            return
        qp, g = host(used["q_prev"]), host(out)
        scale = max(1.0, float(np.max(np.abs(g))))
        m = used["m"]
        if rec["type"] == "full":
            qo, _ = fv.hdm_step(prob, qp)
            e = rel(g, qo)
            assert e <= tol, (k, "full", e)
            st["eps_o"] = None
            st["basis_used"] = ((host(used["Phi"])[: m * n].reshape(m, n).T.copy(), host(used["psi"]))
                                if m > 0 else None)
        else:
            hat, tilde, _ = used["samples"].export()
            hat, tilde = host(hat), host(tilde)
            if st["sets_o"] is not None:
                assert np.array_equal(hat, st["sets_o"]["hat"]) and np.array_equal(tilde, st["sets_o"]["tilde"]), k
            Phi = host(used["Phi"])[: m * n].reshape(m, n).T.copy()
            psi = host(used["psi"])
            norms = []
            ref = step(qp, Phi, psi, hat, tilde, norms=norms)
            assert rec["J"] == ref["J"], (k, rec["J"], ref["J"])
            e = rel(g, ref["gamma"])
            if e > tol:
                assert not gn, (k, "hybrid (Gauss-Newton)", e)
                flips = gate_flips(k, drv.recorder.tapes[k].info()[1], ref["masks"], norms, scale)
                assert flips > 0, (k, "hybrid", e)
                st["ties"].append((k, "gate", flips, e))
                g, e = ref["gamma"], 0.0   # the indicator is compared on the oracle's valid choice
            eg = host(drv.eps)
            itol, ctol = fit_tols(rec["fit_cond"])
            st["cell_tol"] = ctol
            ok, d = indicator_close(eg, ref["eps"], g, tol=itol, cell_tol=ctol)
            if not ok:
                a, b_ = np.sqrt(eg), np.sqrt(ref["eps"])
                worst = np.argsort(np.abs(a - b_))[::-1][:5]
                hm = np.zeros(prob.ncell, bool)
                hm[hat] = True
                print("  indicator mismatch: cells", worst, "in hat", hm[worst], "sqrt eps gpu", a[worst],
                      "oracle", b_[worst], "state diff", (g - ref["gamma"])[worst], "fit cond", rec.get("fit_cond"),
                      "state rel", e, flush=True)
            assert ok, (k, "indicator", d, rec["fit_cond"])
            if st["basis_o"] is not None and st["basis_o"]["m_eff"] == m:
                own = step(qp, st["basis_o"]["Phi"], st["basis_o"]["psi_new"], hat, tilde)
                st["worst_own"] = max(st["worst_own"], rel(host(out), own["gamma"]))
            st["eps_o"] = ref["eps"]
        st["worst"] = max(st["worst"], e)
        st["checked"] += 1

    def on_update(k, rec, s):
        if k < check_from:
            return
        window = [host(x) for x in s["window"]]
        b = pod.pod(window, wl.w, wl.m)
        sg = host(s["sigma"])
        so = b["sigma"]
        assert np.max(np.abs(sg - so)) <= 1e-13 * so[0], (k, "sigma", np.max(np.abs(sg - so)) / so[0])
        me = s["m_eff"]
        if me != b["m_eff"]:
            i = min(me, b["m_eff"])
            assert abs(so[i] / (so[0] * 1e-8) - 1.0) < 1e-9, (k, "m_eff", me, b["m_eff"])
            st["ties"].append((k, "m_eff", me, b["m_eff"]))
        else:
            P = host(s["Phi"])[: me * n].reshape(me, n).T
            Q, _ = np.linalg.qr(P)
            X = b["X"]
            d = np.linalg.norm(Q @ (Q.T @ X) - b["Phi"] @ (b["Phi"].T @ X)) / np.linalg.norm(X)
            assert d <= projector_tol(so, me), (k, "projector", d)
        st["basis_o"] = b
        st["sets_o"] = None
        if s["samples"] is not None:
            eps_o = st["eps_o"]
            if eps_o is None:        # after a full step: the indicator with the basis that step saw
                Phi_u, psi_u = st["basis_used"]
                eps_o, _ = sampling.indicator_full(prob, window[-1], Phi_u, psi_u, hp.floor_rel)
                ok, d = indicator_close(host(s["eps"]), eps_o, window[-1], tol=1e-12)
                assert ok, (k, "indicator (full step)", d)
            sel = sampling.select(prob, eps_o, sampling.RULE_FRACTION, wl.frac, halo=wl.halo)
            hat, tilde, _ = s["samples"].export()
            hat, tilde = host(hat), host(tilde)
            if not (np.array_equal(hat, sel["hat"]) and np.array_equal(tilde, sel["tilde"])):
                # a near tie of the cut: the n_g-th and (n_g+1)-th errors closer
                # (as error norms sqrt(eps)) than the indicator's resolution
                srt = np.sqrt(np.sort(eps_o)[::-1])
                ng = sel["n_g"]
                gap = abs(srt[ng - 1] - srt[ng]) if ng < srt.size else np.inf
                res = st.get("cell_tol", 1e-10) * max(1.0, float(np.max(np.abs(window[-1]))))
                assert gap <= res, (k, "sets", gap, res)
                st["ties"].append((k, "sets", gap))
            else:
                st["sets_o"] = sel

    qT, recs = drv.run(dev(q0), steps, on_step=on_step, on_update=on_update)
    print(f"  {steps} steps, {st['checked']} checked: max rel diff {st['worst']:.2e} (oracle's own basis: "
          f"{st['worst_own']:.2e}); ties {st['ties']}", flush=True)
    assert st["checked"] == steps - check_from + 1
    return prob, q0, host(qT), recs, st


def test_burgers1d_1k_trajectory():
    need_gpu()
    print_case("trajectory burgers1d_1k, 200 steps, resync every step")
    wl = W.WORKLOADS["burgers1d_1k"]
    prob, q0, qT, recs, st = run_resync(wl, 0, wl.steps)
    assert sum(t == "full" for t in st["types"]) == 25
    qH = q0.copy()
    for _ in range(wl.steps):
        qH, _ = fv.hdm_step(prob, qH)
    print(f"  e_T against the full model {arom.relative_l1_error(qT, qH):.3e}", flush=True)


def test_burgers1d_256k_trajectory_window():
    """Config 1's size (262144 cells, m 20, w 30, 5 %): the first 20 hybrid
    steps after the first basis, every one checked against the oracle (the
    full-mesh 1D sweeps run over many 1024-cell tiles here)."""
    need_gpu()
    print_case("trajectory burgers1d_256k, steps w..w+20, resync every step")
    wl = W.WORKLOADS["burgers1d_256k"]
    prob, q0, qT, recs, st = run_resync(wl, 0, wl.w + 21, check_from=wl.w - 1)
    assert sum(t == "hybrid" for t in st["types"]) >= 15


def test_burgers2d_small_trajectory():
    need_gpu()
    print_case("trajectory burgers2d 48x40")
    wl = W.WORKLOADS["burgers2d_1024"].resized(48, 40, m=10)
    prob, q0, qT, recs, st = run_resync(wl, 1, wl.w + 30)
    assert any(t == "hybrid" for t in st["types"])


def test_euler2d_small_trajectory():
    need_gpu()
    print_case("trajectory euler2d 24x20")
    wl = W.WORKLOADS["euler2d_512"].resized(24, 20, m=8)
    prob, q0, qT, recs, st = run_resync(wl, 2, wl.w + 25)
    assert any(t == "hybrid" for t in st["types"])


def test_burgers1d_1k_trajectory_gauss_newton():
    """Alg. 1 with Gauss-Newton subiterations (rom_hybrid_step_gn in the
    driver), resynchronised at every step against the oracle's Gauss-Newton
    step: 1D Burgers 1024 cells, 120 steps."""
    need_gpu()
    print_case("trajectory burgers1d_1k with Gauss-Newton subiterations, 120 steps, resync every step")
    wl = W.WORKLOADS["burgers1d_1k"]
    prob, q0, qT, recs, st = run_resync(wl, 0, 120, gn=True)
    assert sum(r["type"] == "hybrid" for r in recs) > 60
    assert st["worst"] <= 1e-12


def test_burgers2d_small_trajectory_gauss_newton():
    need_gpu()
    print_case("trajectory burgers2d 40x36 (m = 10) with Gauss-Newton subiterations, resync every step")
    wl = W.WORKLOADS["burgers2d_1024"].resized(40, 36, m=10)
    prob, q0, qT, recs, st = run_resync(wl, 1, wl.w + 30, gn=True)
    assert st["worst"] <= 1e-12
