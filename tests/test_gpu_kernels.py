"""GPU parity of the HIP kernels against the FP64 oracle (called through the
C ABI).  Residual and filter are computed in the oracle's operation order,
so they are compared bit for bit; the Newton solve, selection, basis and fit
to the tolerances stated in each test."""
import numpy as np
import pytest

import workloads as W
from oracle import fv, hybrid, pod, sampling

from gpu_common import (CASES, case, ctx_for, dev, host, indicator_close, need_gpu, print_case,
                        projector_tol, rel, torch)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", list(CASES))
def test_residual_bitwise(name):
    need_gpu()
    print_case("residual", name)
    wl, prob, q0 = case(name, 1)
    q1, _ = fv.hdm_step(prob, q0)
    rng = np.random.default_rng(2)
    qp = q0 * (1 + 1e-3 * rng.standard_normal(q0.size))
    ctx = ctx_for(prob)
    R = host(ctx.residual(dev(q1), dev(qp)))
    Ro = fv.residual(prob, q1, qp)
    assert np.array_equal(R, Ro), np.max(np.abs(R - Ro))


@pytest.mark.parametrize("name,nx,ny", [("burgers2d_1024", 1100, 1001), ("euler2d_512", 520, 505)])
def test_residual_column_bands_bitwise(name, nx, ny):
    """Meshes large enough for the residual's column-band form (2D Burgers
    above 2^20 cells: 4 rows per thread; 2D Euler from 2^18 cells: 2 rows),
    with a ragged last band and a partial last block of columns: the same
    bits as the oracle."""
    import dataclasses
    need_gpu()
    print_case("residual (column bands)", name, nx, ny)
    wl = dataclasses.replace(W.WORKLOADS[name], nx=nx, ny=ny)
    prob, q0 = W.make(wl, 3)
    rng = np.random.default_rng(4)
    q = q0 * (1 + 1e-3 * rng.standard_normal(q0.size))
    qp = q0 * (1 + 1e-3 * rng.standard_normal(q0.size))
    ctx = ctx_for(prob, m_max=1, w_max=2)
    R = host(ctx.residual(dev(q), dev(qp)))
    Ro = fv.residual(prob, q, qp)
    assert np.array_equal(R, Ro), np.max(np.abs(R - Ro))


def test_stream_add_reference():
    """The streaming reference of the bandwidth measurements adds exactly
    (a ragged element count)."""
    need_gpu()
    print_case("hs_stream_add")
    wl, prob, q0 = case("burgers2d", 0)
    ctx = ctx_for(prob, m_max=1, w_max=2)
    rng = np.random.default_rng(7)
    a, b = rng.standard_normal(100003), rng.standard_normal(100003)
    out = dev(np.zeros(100003))
    ctx.stream_add(dev(a), dev(b), out)
    assert np.array_equal(host(out), a + b)


@pytest.mark.parametrize("name", list(CASES))
def test_jvp_matches_oracle_jacobian(name):
    need_gpu()
    print_case("jvp", name)
    wl, prob, q0 = case(name, 2)
    rng = np.random.default_rng(3)
    q = q0 * (1 + 0.01 * rng.standard_normal(q0.size))
    v = rng.standard_normal(q0.size)
    ctx = ctx_for(prob)
    Jv = host(ctx.jvp(dev(q), dev(v)))
    Jo = fv.jacobian(prob, q) @ v
    assert rel(Jv, Jo) < 1e-14


@pytest.mark.parametrize("name", list(CASES))
def test_hdm_step_matches_oracle(name):
    need_gpu()
    print_case("hdm_step", name)
    wl, prob, q0 = case(name, 0)
    ctx = ctx_for(prob)
    q = q0
    qg = dev(q0)
    for k in range(3):
        qo, _ = fv.hdm_step(prob, q)
        qn, info = ctx.hdm_step(dev(q))
        qn = host(qn)
        assert rel(qn, qo) < 1e-12, (k, rel(qn, qo), info)
        # property at any size: the GPU state solves the oracle's residual
        assert np.max(np.abs(fv.residual(prob, qn, q))) <= 2 * fv.newton_tol(q)
        q = qo


@pytest.mark.parametrize("name", list(CASES))
def test_sample_select_bit_exact(name):
    need_gpu()
    print_case("sample_select", name)
    wl, prob, q0 = case(name, 3)
    rng = np.random.default_rng(4)
    eps = rng.random(prob.ncell) ** 6
    eps[rng.random(prob.ncell) < 0.3] = 0.0
    eps[10:20] = eps[100]                  # ties at various places
    eps[200:260] = 0.5
    ctx = ctx_for(prob)
    # fractions above and below the positive share (the cap n_g <= #{eps > 0}),
    # then an error field without a positive entry
    cases = [(eps, frac) for frac in (0.0, 0.01, wl.frac, 0.3, 1.0)] + [(np.zeros(prob.ncell), 0.3)]
    for eps, frac in cases:
        o = sampling.select(prob, eps, sampling.RULE_FRACTION, frac, halo=2)
        s = ctx.sample_select(dev(eps), frac, halo=2)
        c = s.counts()
        hat, tilde, mask = s.export()
        assert c["n_g"] == o["n_g"] and c["n_s"] == o["hat"].size and c["l"] == o["tilde"].size
        assert np.array_equal(host(hat), o["hat"])
        assert np.array_equal(host(tilde), o["tilde"])
        assert np.array_equal(host(mask).astype(bool), o["mask"])


def test_samples_set_derives_ring():
    need_gpu()
    wl, prob, q0 = case("burgers2d")
    rng = np.random.default_rng(5)
    hat = np.flatnonzero(rng.random(prob.ncell) < 0.05).astype(np.int32)
    mask = np.zeros(prob.ncell, bool)
    mask[hat] = True
    ctx = ctx_for(prob)
    s = ctx.samples_set(dev(hat))
    h, t, m = s.export()
    assert np.array_equal(host(h), hat)
    assert np.array_equal(host(t), np.flatnonzero(sampling.neighbours(prob, mask)))


def window(prob, q0, w, extra=1):
    snaps = [q0]
    for _ in range(w - 1 + extra):
        snaps.append(fv.hdm_step(prob, snaps[-1])[0])
    return snaps


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("w,m,first", [(12, 8, False), (12, 8, True), (30, 20, False), (48, 32, False),
                                       (60, 40, False)])
def test_basis_update_matches_oracle(name, w, m, first):
    """Windows padded to 16, 32, 48 and 64 columns (every instantiation of the
    window passes), the first update (w snapshots) and the later ones (w + 1)."""
    need_gpu()
    print_case("basis_update", name, w, m, first)
    wl, prob, q0 = case(name, 1)
    snaps = window(prob, q0, w, extra=0 if first else 1)
    o = pod.pod(snaps, w, m)
    ctx = ctx_for(prob)
    Phi = torch.zeros(m * prob.n, dtype=torch.float64, device="cuda")
    psi = ctx.empty()
    sig = torch.zeros(w, dtype=torch.float64, device="cuda")
    me = ctx.basis_update([dev(s) for s in snaps], w, m, Phi, psi, sig)
    # the window means round the exact sum on both sides: equal to the bit
    assert np.array_equal(host(psi), o["psi_new"])
    sg, so = host(sig), o["sigma"]
    # sigma from the triangular factor of X: absolute accuracy of a few eps sigma_0
    print(f"  m_eff {me}, sigma err {np.max(np.abs(sg - so)) / so[0]:.2e} sigma_0, cut {so[me - 1] / so[0]:.1e}")
    assert np.max(np.abs(sg - so)) <= 1e-13 * so[0]
    assert me == o["m_eff"]
    P = host(Phi).reshape(m, prob.n)[:me].T
    # Phi = X V diag(1/sigma): the rounding of X V (eps ||X||) leaves an
    # orthogonality error of order eps sigma_0 / sigma_{m_eff-1}
    orth = np.max(np.abs(P.T @ P - np.eye(me)))
    assert orth < max(1e-13, 20 * 2.2e-16 * so[0] / so[me - 1]), orth
    X = o["X"]
    Q, _ = np.linalg.qr(P)                 # orthogonal projector onto span(Phi)
    Pg = Q @ (Q.T @ X)
    Po = o["Phi"] @ (o["Phi"].T @ X)
    tol = projector_tol(so, me)
    assert np.linalg.norm(Pg - Po) <= tol * np.linalg.norm(X), (np.linalg.norm(Pg - Po) / np.linalg.norm(X), tol)


@pytest.mark.parametrize("name", list(CASES))
def test_filter_matches_oracle(name):
    need_gpu()
    print_case("filter", name)
    wl, prob, q0 = case(name, 2)
    q1, _ = fv.hdm_step(prob, q0)
    rng = np.random.default_rng(6)
    noisy = q1 + 1e-3 * np.abs(q1).max() * rng.standard_normal(q1.size) * (rng.random(q1.size) < 0.1)
    ctx = ctx_for(prob)
    out, info = ctx.filter(dev(noisy), dev(q0))
    ref = hybrid.spatial_filter(prob, noisy, q0, hybrid.HybridParams())
    assert info["filter_passes"] > 0
    assert np.array_equal(host(out), ref), np.max(np.abs(host(out) - ref))


@pytest.mark.parametrize("name", list(CASES))
def test_indicator_full_matches_oracle(name):
    need_gpu()
    print_case("indicator_full", name)
    wl, prob, q0 = case(name, 4)
    w, m = 10, 6
    snaps = window(prob, q0, w)
    o = pod.pod(snaps, w, m)
    g = fv.hdm_step(prob, snaps[-1])[0]
    me = o["m_eff"]
    ctx = ctx_for(prob)
    Phi = dev(np.ascontiguousarray(o["Phi"].T).reshape(-1))
    eps, y = ctx.indicator_full(dev(g), Phi, dev(o["psi_new"]), me)
    eo, yo = sampling.indicator_full(prob, g, o["Phi"], o["psi_new"])
    assert rel(host(y), yo) < 1e-12
    ok, d = indicator_close(host(eps), eo, g)
    assert ok, d


@pytest.mark.parametrize("name", list(CASES))
def test_hybrid_step_matches_oracle(name):
    need_gpu()
    print_case("rom_hybrid_step", name)
    wl, prob, q0 = case(name, 0)
    w, m = 12, 8
    snaps = window(prob, q0, w)
    o = pod.pod(snaps, w, m)
    Phi_o, psi = o["Phi"], o["psi_new"]
    me = o["m_eff"]
    g = snaps[-1]
    eps, _ = sampling.indicator_full(prob, g, Phi_o, psi)
    sel = sampling.select(prob, eps, sampling.RULE_FRACTION, wl.frac)
    ref = hybrid.hybrid_step(prob, g, Phi_o, psi, sel["hat"], sel["tilde"])
    ctx = ctx_for(prob)
    s = ctx.samples_set(dev(sel["hat"]))
    Phi = dev(np.ascontiguousarray(Phi_o.T).reshape(-1))
    eps_g = ctx.empty(prob.ncell)
    y_g = ctx.empty(me)
    out, info = ctx.rom_hybrid_step(dev(g), Phi, dev(psi), me, s, eps=eps_g, y=y_g)
    print("  info", info, "J_oracle", ref["J"], flush=True)
    assert info["subiters"] == ref["J"]
    assert rel(host(y_g), ref["y"]) < 1e-10
    assert rel(host(out), ref["gamma"]) < 1e-12, rel(host(out), ref["gamma"])
    ok, d = indicator_close(host(eps_g), ref["eps"], ref["gamma"], tol=1e-12, cell_tol=1e-10)
    assert ok, d


@pytest.mark.parametrize("name", list(CASES))
def test_small_pinv_equals_lds_pinv(name):
    """The one-wave register pseudo-inverse of the fit (m <= 8) takes the
    LDS routine's rotations in the same order: the hybrid step is the same bit
    for bit with either, over several basis widths."""
    need_gpu()
    wl, prob, q0 = case(name, 0)
    w = 12
    snaps = window(prob, q0, w)
    ctx = ctx_for(prob)
    g = snaps[-1]
    for m in (1, 3, 5, 8):
        o = pod.pod(snaps, w, m)
        Phi_o, psi, me = o["Phi"], o["psi_new"], o["m_eff"]
        print_case("small pinv", name, "m", m, "m_eff", me)
        eps, _ = sampling.indicator_full(prob, g, Phi_o, psi)
        sel = sampling.select(prob, eps, sampling.RULE_FRACTION, wl.frac)
        s = ctx.samples_set(dev(sel["hat"]))
        Phi = dev(np.ascontiguousarray(Phi_o.T).reshape(-1))
        outs = []
        for on in (True, False):
            ctx.set_small_pinv(on)
            y_g = ctx.empty(me)
            out, info = ctx.rom_hybrid_step(dev(g), Phi, dev(psi), me, s, y=y_g)
            outs.append((out, y_g, info))
        ctx.set_small_pinv(True)
        (o1, y1, i1), (o2, y2, i2) = outs
        assert torch.equal(o1, o2)
        assert torch.equal(y1, y2)
        assert i1["subiters"] == i2["subiters"]
        assert i1["fit_rank"] == i2["fit_rank"] and i1["fit_cond"] == i2["fit_cond"]


@pytest.mark.parametrize("name", list(CASES))
def test_tiled_sweeps_equal_list_sweeps(name):
    """The LDS-tiled relaxation (several sweeps per launch) and the one-sweep
    compact-list relaxation give the same iterates bit for bit: full and
    sampled Newton solves, and the transposed solve of the adjoint, with tiles
    where they are dense and with tiles forced on every sampled set."""
    need_gpu()
    print_case("tiled sweeps", name)
    wl, prob, q0 = case(name, 0)
    w, m = 12, 8
    snaps = window(prob, q0, w)
    o = pod.pod(snaps, w, m)
    g = snaps[-1]
    eps, _ = sampling.indicator_full(prob, g, o["Phi"], o["psi_new"])
    sel = sampling.select(prob, eps, sampling.RULE_FRACTION, wl.frac)
    Phi = dev(np.ascontiguousarray(o["Phi"].T).reshape(-1))
    outs = []
    for tiled in (False, True, "always"):     # list; tiles where dense; tiles on every set
        ctx = ctx_for(prob)
        ctx.set_tiled_sweeps(tiled)
        full, fi = ctx.hdm_step(dev(g))
        s = ctx.samples_set(dev(sel["hat"]))
        hyb, hi = ctx.rom_hybrid_step(dev(g), Phi, dev(o["psi_new"]), o["m_eff"], s)
        lam = dev(np.random.default_rng(2).standard_normal(prob.n))
        adj, ai = ctx.hdm_step_adjoint(full, lam)
        print("  tiled", tiled, "sweeps", fi["lin_sweeps"], hi["lin_sweeps"], ai["lin_sweeps"], flush=True)
        outs.append((full, hyb, adj, fi["lin_sweeps"], hi["lin_sweeps"]))
    a0, b0, c0, f0, h0 = outs[0]
    for a1, b1, c1, f1, h1 in outs[1:]:
        assert (f0, h0) == (f1, h1)
        assert torch.equal(a0, a1)
        assert torch.equal(b0, b1)
        assert torch.equal(c0, c1)


@pytest.mark.parametrize("name", list(CASES))
def test_sample_select_rre_bit_exact(name):
    """The RRE rule (eq. rre, exact fixed-point sums): n_g, hat-S and
    tilde-S equal the oracle's for several delta, on a real indicator and on
    an indicator with many exact ties."""
    need_gpu()
    print_case("sample_select RRE", name)
    import paper_2301_01718_amd as hs
    wl, prob, q0 = case(name, 2)
    w, m = 10, 6
    snaps = window(prob, q0, w)
    o = pod.pod(snaps, w, m)
    g = fv.hdm_step(prob, snaps[-1])[0]
    eps_real, _ = sampling.indicator_full(prob, g, o["Phi"], o["psi_new"])
    rng = np.random.default_rng(4)
    eps_ties = rng.integers(0, 6, prob.ncell).astype(float) * 0.125 * rng.choice([1.0, 2.0 ** -40], prob.ncell)
    ctx = ctx_for(prob)
    for eps in (eps_real, eps_ties):
        for delta in (0.3, 0.8, 0.9, 0.99, 1.0, 1.5):
            s = ctx.sample_select(dev(eps), 0.0, halo=wl.halo, rule=hs.RULE_RRE, delta=delta)
            o_sel = sampling.select(prob, eps, sampling.RULE_RRE, delta=delta, halo=wl.halo)
            hat, tilde, _ = s.export()
            print(f"  delta {delta}: n_g {s.counts()['n_g']} oracle {o_sel['n_g']}", flush=True)
            assert s.counts()["n_g"] == o_sel["n_g"]
            assert np.array_equal(host(hat), o_sel["hat"]) and np.array_equal(host(tilde), o_sel["tilde"])


def test_basis_update_async_equals_sync():
    """basis_update_async + basis_update_finish give the synchronous result
    bit for bit, with a sample_select run on the main stream in between; a
    second update is rejected while one is in flight."""
    need_gpu()
    print_case("basis_update_async")
    import paper_2301_01718_amd as hs
    wl, prob, q0 = case("burgers2d", 1)
    w, m = 12, 8
    snaps = [dev(s) for s in window(prob, q0, w)]
    eps = dev(np.random.default_rng(0).random(prob.ncell))
    ctx = ctx_for(prob)
    outs = []
    for mode in ("sync", "async"):
        P = torch.zeros(m * prob.n, dtype=torch.float64, device="cuda")
        psi = ctx.empty()
        sig = torch.zeros(w, dtype=torch.float64, device="cuda")
        if mode == "sync":
            me = ctx.basis_update(snaps, w, m, P, psi, sig)
            s = ctx.sample_select(eps, wl.frac, halo=wl.halo)
        else:
            ctx.basis_update_async(snaps, w, m, P, psi, sig)
            with pytest.raises(hs.HsError):
                ctx.basis_update(snaps, w, m, P, psi, sig)
            s = ctx.sample_select(eps, wl.frac, halo=wl.halo)
            me = ctx.basis_update_finish()
        outs.append((me, P.clone(), psi.clone(), sig.clone(), [host(x) for x in s.export()[:2]]))
    (m0, P0, p0, s0, h0), (m1, P1, p1, s1, h1) = outs
    assert m0 == m1 and torch.equal(P0, P1) and torch.equal(p0, p1) and torch.equal(s0, s1)
    assert all(np.array_equal(a, b) for a, b in zip(h0, h1))
