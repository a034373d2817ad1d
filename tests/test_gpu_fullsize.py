"""Parity at the benchmark's full size: 2D Burgers, 1024 x 1024 cells, m = 32,
w = 48, 5 % sampled with a 2-cell halo.

test_full_size_parity: element by element against the oracle, on inputs that
come only from the seeded generator and the oracle.  The window is w + 1
translates of the seeded initial state (exact solutions of linear advection:
a moving front, produced by index shifts, none of the method's arithmetic).
  * basis_update vs the oracle POD of that window: psi to 1e-15, m_eff equal,
    sigma^2 to 1e-13 sigma_0^2, projector within the Davis-Kahan bound;
  * sample_select on the oracle's indicator: hat-S and tilde-S bit for bit;
  * rom_hybrid_step with the oracle basis and sets vs the oracle step: 1e-12
    relative, equal subiteration count J;
  * hs_filter on a seeded noisy state vs the oracle filter: bit for bit;
  * hdm_step: the oracle residual (eq. hdm) of the GPU state is within the
    Newton tolerance (the oracle's sparse direct solve takes minutes at
    10^6 cells, the residual is one pass).

test_bench_configuration_properties: the benchmark's own trajectory and
launch configuration (the steps bench.py times), checked through properties
that hold at any size: bases orthonormal to the method-of-snapshots bound, the sampled-set invariants (G holds
the n_g largest errors, hat-S is G dilated, tilde-S its face ring), finite
hybrid snapshots whose subiteration counts stay within J_max, and full steps
whose oracle residual is within the Newton tolerance."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fv, hybrid, pod, sampling

from gpu_common import ctx_for, dev, host, need_gpu, print_case, projector_tol, rel, torch, validate_filter

pytestmark = pytest.mark.gpu

WL = W.WORKLOADS["burgers2d_1024"]


def translated_window(prob, q0, w):
    g = q0.reshape(prob.ny, prob.nx)
    return [np.roll(np.roll(g, k, axis=1), k // 2, axis=0).reshape(-1).copy() for k in range(w + 1)]


def test_full_size_parity():
    need_gpu()
    print_case("full size burgers2d_1024, independent inputs")
    prob, q0 = W.make(WL, 0)
    w, m = WL.w, WL.m
    snaps = translated_window(prob, q0, w)
    ctx = ctx_for(prob, m_max=m, w_max=w)

    # basis
    b = pod.pod(snaps, w, m)
    me = b["m_eff"]
    Pg = torch.zeros(m * prob.n, dtype=torch.float64, device="cuda")
    psig, sg = ctx.empty(), torch.zeros(w, dtype=torch.float64, device="cuda")
    me_g = ctx.basis_update([dev(s) for s in snaps], w, m, Pg, psig, sg)
    assert me_g == me
    assert np.array_equal(host(psig), b["psi_new"])
    so = b["sigma"]
    ds = np.max(np.abs(host(sg) - so)) / so[0]
    P = host(Pg)[: me * prob.n].reshape(me, prob.n).T
    orth = np.max(np.abs(P.T @ P - np.eye(me)))
    X = b["X"]
    Q, _ = np.linalg.qr(P)                 # orthogonal projector onto span(Phi)
    d = np.linalg.norm(Q @ (Q.T @ X) - b["Phi"] @ (b["Phi"].T @ X)) / np.linalg.norm(X)
    tol = projector_tol(so, me)
    print(f"  basis: m_eff {me}, sigma err {ds:.1e} sigma_0, projector difference {d:.2e} (bound {tol:.2e}), "
          f"orthogonality {orth:.1e}", flush=True)
    assert ds <= 1e-13
    assert d <= tol
    assert orth < max(1e-13, 20 * 2.2e-16 * so[0] / so[me - 1])
    del Pg, P, Q

    # sampled sets from the oracle's indicator
    g = snaps[-1]
    psi = b["psi_new"]
    eps, _ = sampling.indicator_full(prob, g, b["Phi"], psi)
    sel = sampling.select(prob, eps, sampling.RULE_FRACTION, WL.frac, halo=WL.halo)
    s = ctx.sample_select(dev(eps), WL.frac, WL.halo)
    hat, tilde, _ = s.export()
    assert np.array_equal(host(hat), sel["hat"]) and np.array_equal(host(tilde), sel["tilde"])
    print(f"  sets: n_s {sel['hat'].size}, l {sel['tilde'].size}", flush=True)

    # hybrid step from the oracle's basis and sets
    Phi_rows = dev(np.ascontiguousarray(b["Phi"].T).reshape(-1))
    out, info = ctx.rom_hybrid_step(dev(g), Phi_rows, dev(psi), me, s)
    ref = hybrid.hybrid_step(prob, g, b["Phi"], psi, sel["hat"], sel["tilde"])
    e = rel(host(out), ref["gamma"])
    print(f"  hybrid step: rel error {e:.2e}, J gpu {info['subiters']} oracle {ref['J']}", flush=True)
    assert e < 1e-12 and info["subiters"] == ref["J"]
    del Phi_rows

    # filter on a seeded noisy state
    rng = np.random.default_rng(11)
    noisy = g + 1e-3 * np.abs(g).max() * rng.standard_normal(g.size) * (rng.random(g.size) < 0.05)
    fo, finfo = ctx.filter(dev(noisy), dev(snaps[-2]))
    fr = hybrid.spatial_filter(prob, noisy, snaps[-2], hybrid.HybridParams())
    print(f"  filter: {finfo['filter_passes']} passes, max diff {np.max(np.abs(host(fo) - fr)):.1e}", flush=True)
    assert finfo["filter_passes"] > 0 and np.array_equal(host(fo), fr)

    # full HDM step: the oracle residual of the GPU state
    full, hinfo = ctx.hdm_step(dev(g))
    R = fv.residual(prob, host(full), g)
    tol = fv.newton_tol(g)
    print(f"  hdm step: newton {hinfo['newton_iters']}, oracle ||R||_inf {np.max(np.abs(R)):.2e} "
          f"(tolerance {tol:.2e})", flush=True)
    assert hinfo["newton_iters"] >= 1 and np.max(np.abs(R)) <= tol


def face_ring(prob, mask):
    g = mask.reshape(prob.ny, prob.nx)
    nb = np.zeros_like(g)
    for ax in (0, 1):
        for sh in (1, -1):
            nb |= np.roll(g, sh, axis=ax)
    return (nb & ~g).reshape(-1)


def test_bench_configuration_properties():
    need_gpu()
    print_case("full size burgers2d_1024, bench trajectory properties")
    import paper_2301_01718_amd.driver as D
    prob, q0 = W.make(WL, 0)
    cfg = D.AromConfig(w=WL.w, m=WL.m, z=WL.z, fraction=WL.frac, halo=WL.halo)
    drv = D.Arom(prob, cfg)
    k0 = WL.z * math.ceil((WL.w + 2) / WL.z)
    last = k0 + 2 + 16                                  # setup, 2 warm-up and 16 timed steps
    n_g = math.ceil(WL.frac * prob.ncell)
    seen = {"hybrid": 0, "full": 0, "update": 0}

    def on_step(k, rec, used, out):
        if k < k0:
            return
        o = host(out)
        assert np.all(np.isfinite(o)), k
        if rec["type"] == "hybrid":
            seen["hybrid"] += 1
            assert 1 <= rec["J"] <= cfg.jmax, (k, rec["J"])
        else:
            seen["full"] += 1
            qp = host(used["q_prev"])
            assert np.max(np.abs(fv.residual(prob, o, qp))) <= fv.newton_tol(qp), k

    def on_update(k, rec, st):
        if k < k0:
            return
        seen["update"] += 1
        me = st["m_eff"]
        P = host(st["Phi"])[: me * prob.n].reshape(me, prob.n)
        sig = host(st["sigma"])[:me]
        # Phi = X V diag(1/sigma) is orthonormal to about
        # eps sigma_0 / min(sigma_i, sigma_j) (the rounding of X V)
        bound = np.maximum(20 * 2.2e-16 * sig[0] / np.minimum.outer(sig, sig), 1e-14)
        assert (np.abs(P @ P.T - np.eye(me)) <= bound).all(), k
        if st["samples"] is not None:
            hat, tilde, _ = st["samples"].export()
            hat, tilde = host(hat), host(tilde)
            eps = host(st["eps"])
            ng = rec["n_g"]
            assert ng == min(n_g, int(np.count_nonzero(eps > 0))), k
            hm = np.zeros(prob.ncell, dtype=bool)
            hm[hat] = True
            # G = the n_g largest errors: every error above the cut is sampled,
            # and hat-S lies inside the dilation of the cells at or above it
            cut = np.sort(eps)[-ng]
            assert hm[eps > cut].all(), k
            assert not (hm & ~sampling.dilate(prob, eps >= cut, WL.halo)).any(), k
            assert np.array_equal(np.flatnonzero(face_ring(prob, hm)), tilde), k
            assert np.all(np.diff(hat) > 0), k

    drv.start(dev(q0), WL.steps)
    while drv.k < last:
        drv.advance(on_step, on_update)
    print(f"  steps {k0}..{last}: {seen}", flush=True)
    assert seen["hybrid"] >= 16 and seen["full"] >= 1 and seen["update"] >= 16


WL3 = W.WORKLOADS["euler2d_512"]


def test_euler_full_size_parity():
    """Config 3's size (2D Euler 512 x 512, m 40, w 60, 8 %): the basis of a
    window of translates (sigma, m_eff, span), the sets from the oracle's
    indicator (bit for bit), one hybrid step on the oracle's basis and sets
    (1e-12, equal J) and a full step checked by the oracle's residual."""
    need_gpu()
    print_case("full size euler2d_512, independent inputs")
    prob, q0 = W.make(WL3, 0)
    w, m = WL3.w, WL3.m
    g3 = q0.reshape(prob.ncomp, prob.ny, prob.nx)
    snaps = [np.roll(np.roll(g3, k, axis=2), k // 2, axis=1).reshape(-1).copy() for k in range(w + 1)]
    ctx = ctx_for(prob, m_max=m, w_max=w)
    b = pod.pod(snaps, w, m)
    me = b["m_eff"]
    Pg = torch.zeros(m * prob.n, dtype=torch.float64, device="cuda")
    psig, sg = ctx.empty(), torch.zeros(w, dtype=torch.float64, device="cuda")
    me_g = ctx.basis_update([dev(s) for s in snaps], w, m, Pg, psig, sg)
    so = b["sigma"]
    ds = np.max(np.abs(host(sg) - so)) / so[0]
    P = host(Pg)[: me * prob.n].reshape(me, prob.n).T
    Q, _ = np.linalg.qr(P)
    X = b["X"]
    d = np.linalg.norm(Q @ (Q.T @ X) - b["Phi"] @ (b["Phi"].T @ X)) / np.linalg.norm(X)
    print(f"  basis: m_eff {me_g}/{me}, sigma err {ds:.1e} sigma_0, projector difference {d:.1e}", flush=True)
    assert me_g == me and ds <= 1e-13 and d <= projector_tol(so, me)
    assert np.array_equal(host(psig), b["psi_new"])
    del Pg, P, Q

    g = snaps[-1]
    psi = b["psi_new"]
    eps, _ = sampling.indicator_full(prob, g, b["Phi"], psi)
    sel = sampling.select(prob, eps, sampling.RULE_FRACTION, WL3.frac, halo=WL3.halo)
    s = ctx.sample_select(dev(eps), WL3.frac, WL3.halo)
    hat, tilde, _ = s.export()
    assert np.array_equal(host(hat), sel["hat"]) and np.array_equal(host(tilde), sel["tilde"])
    print(f"  sets: n_s {sel['hat'].size}, l {sel['tilde'].size}", flush=True)

    # the step is taped so that its filter passes (order, kept cells) can be
    # checked: the residual-gated filter acts on shocks here, and a gate
    # decided by a residual-norm difference at the rounding level of the
    # step's inputs may go either way (both correct); every flag is checked
    # on the oracle's side pass by pass, and the states compared on the same
    # flags
    from paper_2301_01718_amd import TAPE_RECORD
    Phi_rows = dev(np.ascontiguousarray(b["Phi"].T).reshape(-1))
    tape = ctx.tape()
    out, info = ctx.rom_hybrid_step_taped(dev(g), Phi_rows, dev(psi), me, tape, TAPE_RECORD, samples=s)
    J, passes = tape.info()
    print(f"  gpu hybrid step: J {info['subiters']}, newton {info['newton_iters']}, filter passes {len(passes)}",
          flush=True)
    nof = hybrid.hybrid_step(prob, g, b["Phi"], psi, sel["hat"], sel["tilde"], hybrid.HybridParams(filter_orders=()))
    assert J == nof["J"]
    pre = nof["gamma"]
    ref, ties = validate_filter(prob, pre, g, [(n, host(mk)) for n, mk in passes])
    e = rel(host(out), ref)
    print(f"  hybrid step: rel error {e:.2e} on the same filter flags ({ties} tied flags), J {J}", flush=True)
    assert e < 1e-12
    del Phi_rows

    full, hinfo = ctx.hdm_step(dev(g))
    R = fv.residual(prob, host(full), g)
    tol = fv.newton_tol(g)
    print(f"  hdm step: newton {hinfo['newton_iters']}, oracle ||R||_inf {np.max(np.abs(R)):.2e} "
          f"(tolerance {tol:.2e})", flush=True)
    assert hinfo["newton_iters"] >= 1 and np.max(np.abs(R)) <= tol

