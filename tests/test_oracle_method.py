"""Pins of the oracle's sampling, POD, filter, hybrid step and Algorithm-1
schedule (no GPU).  Each check is fixed by the paper or by mathematics
independent of the oracle's own code: brute-force orderings and set
operations, planted SVDs, Eckart-Young, the Shapiro transfer function, the
"all cells sampled = full HDM" and exact-span fixed points, and the closed
form of the step schedule."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import arom, fv, hybrid, pod, sampling

HERE = os.path.dirname(__file__)


# ---------------------------------------------------------------- paper parameters

def test_defaults_equal_paper_parameters():
    pp = json.load(open(os.path.join(HERE, "golden", "paper_parameters.json")))
    hp = hybrid.HybridParams()
    assert hp.eps_y == pp["eps_y"]["value"] and hp.jmax == pp["jmax"]["value"]
    assert hp.eps_f == pp["eps_f"]["value"] and hp.jfmax == pp["jfmax"]["value"]
    assert [2 * n for n in hp.filter_orders] == pp["filter_orders"]["value"]
    assert W.GAMMA == pp["gamma"]["value"]


# ---------------------------------------------------------------- selection

def brute_select(prob, eps, ng, halo):
    order = sorted(range(prob.ncell), key=lambda i: (-eps[i], i))
    G = order[:ng]
    nx, ny = prob.nx, prob.ny
    per = prob.bc == W.BC_PERIODIC
    hat = set()
    for c in G:
        i, j = c % nx, c // nx
        for dj in (range(-halo, halo + 1) if ny > 1 else [0]):
            for di in range(-halo, halo + 1):
                ii, jj = i + di, j + dj
                if per:
                    ii, jj = ii % nx, jj % ny
                elif not (0 <= ii < nx and 0 <= jj < ny):
                    continue
                hat.add(ii + nx * jj)
    tilde = set()
    for c in hat:
        i, j = c % nx, c // nx
        nbs = [(i - 1, j), (i + 1, j)] + ([(i, j - 1), (i, j + 1)] if ny > 1 else [])
        for ii, jj in nbs:
            if per:
                ii, jj = ii % nx, jj % ny
            elif not (0 <= ii < nx and 0 <= jj < ny):
                continue
            if ii + nx * jj not in hat:
                tilde.add(ii + nx * jj)
    return G, sorted(hat), sorted(tilde)


@pytest.mark.parametrize("name,nx,ny", [("burgers1d_1k", 97, 1), ("burgers2d_1024", 23, 17),
                                        ("euler2d_512", 19, 21)])
def test_select_matches_brute_force(name, nx, ny):
    wl = W.WORKLOADS[name].resized(nx, ny)
    prob, _ = W.make(wl, 0)
    rng = np.random.default_rng(11)
    eps = rng.random(prob.ncell) ** 4
    eps[rng.random(prob.ncell) < 0.2] = 0.0
    eps[5:9] = eps[40]                      # ties
    out = sampling.select(prob, eps, sampling.RULE_FRACTION, 0.07, halo=2)
    ng = min(math.ceil(0.07 * prob.ncell), int(np.count_nonzero(eps > 0)))
    G, hat, tilde = brute_select(prob, eps, ng, 2)
    assert out["n_g"] == ng and list(out["G"]) == G
    assert list(out["hat"]) == hat and list(out["tilde"]) == tilde
    # set invariants
    s_hat, s_til = set(hat), set(tilde)
    assert set(G) <= s_hat and not (s_hat & s_til)
    assert np.array_equal(out["mask"], np.isin(np.arange(prob.ncell), hat))


def test_select_all_zero_gives_empty_sets():
    prob, _ = W.make(W.WORKLOADS["burgers2d_1024"].resized(8), 0)
    out = sampling.select(prob, np.zeros(prob.ncell), sampling.RULE_FRACTION, 0.5)
    assert out["n_g"] == 0 and out["hat"].size == 0 and out["tilde"].size == 0


def test_rre_rule_is_smallest_count_reaching_delta():
    rng = np.random.default_rng(3)
    eps = rng.random(200) ** 3
    for delta in (0.1, 0.5, 0.8, 0.9, 0.99):
        n = sampling.count_g(eps, sampling.RULE_RRE, delta=delta)
        s = sorted(eps, reverse=True)
        tot = math.fsum(s)
        assert math.fsum(s[:n]) / tot >= delta - 1e-15
        assert math.fsum(s[:n - 1]) / tot < delta + 1e-15


def test_rre_rule_exact_on_the_fixed_point_grid():
    """eq. rre with exact rational sums (brute force) on errors that the
    64-bit encoding represents exactly, including exact hits of delta and
    ties: the rule returns the smallest n with RRE(n) >= delta."""
    from fractions import Fraction
    rng = np.random.default_rng(8)
    for trial in range(40):
        n = int(rng.integers(1, 40))
        ints = rng.integers(0, 9, n) * (1 << int(rng.integers(0, 5)))   # small dyadic integers, many ties
        eps = ints.astype(float) * 2.0 ** -30
        if not np.any(eps > 0):
            continue
        order = sorted(range(n), key=lambda i: (-eps[i], i))
        tot = sum(Fraction(int(v)) for v in ints)
        for delta in (0.25, 0.5, 0.75, 0.8, 0.9, 1.0, float(rng.random())):
            want = None
            acc = Fraction(0)
            for g, i in enumerate(order, start=1):
                acc += int(ints[i])
                if acc / tot >= Fraction(delta):
                    want = g
                    break
            want = min(want, int(np.count_nonzero(eps > 0)))
            assert sampling.count_g(eps, sampling.RULE_RRE, delta=delta) == want, (trial, delta)


def _rre_brute(eps, delta):
    """eq. rre written with Fraction sums (each double converted exactly)."""
    from fractions import Fraction
    order = sorted(range(eps.size), key=lambda i: (-eps[i], i))
    fr = [Fraction(float(v)) for v in eps]
    tot = sum(fr, Fraction(0))
    d = Fraction(float(delta))
    acc = Fraction(0)
    npos = int(np.count_nonzero(eps > 0))
    for g, i in enumerate(order, start=1):
        acc += fr[i]
        if acc >= d * tot:
            return min(g, npos)
    return npos


def test_rre_exact_sums_match_fraction_brute_force():
    """The oracle's integer form of eq. rre equals the definition taken with
    exact rationals, on errors spanning many binades (down to subnormals)."""
    rng = np.random.default_rng(11)
    for trial in range(30):
        n = int(rng.integers(1, 60))
        eps = rng.random(n) * 2.0 ** rng.integers(-1070, 10, n).astype(float)
        eps[rng.random(n) < 0.2] = 0.0
        if trial % 3 == 0:
            eps[: n // 2] = eps[0]                      # ties
        if not np.any(eps > 0):
            continue
        for delta in (1e-12, 0.3, 0.5, 0.9, 0.999999, 1.0, 1.5, float(rng.random())):
            assert sampling.count_g(eps, sampling.RULE_RRE, delta=delta) == _rre_brute(eps, delta), (trial, delta)


def test_exact_dyadic_decomposition():
    from fractions import Fraction
    vals = [0.0, 3.0, 1.5, 2.0 ** -70, 1.0, 5e-324, 0.1]
    k, e = sampling.exact_dyadic(vals)
    for v, ki in zip(vals, k):
        assert Fraction(ki) * Fraction(2) ** e == Fraction(v)


def _fixed_point_count(eps, delta):
    """The library's 64-bit encoding of eq. rre (a model of its documented
    arithmetic, for comparison with the exact rule): q = floor(eps 2^(63 - e_max))
    with 2^e_max <= max eps < 2^(e_max + 1); S >= delta T decided on q;
    delta >= 1 gives every positive cell."""
    npos = int(np.count_nonzero(eps > 0))
    if npos == 0:
        return 0
    if delta >= 1.0:
        return npos
    emax = math.frexp(float(np.max(eps)))[1] - 1
    q = [int(math.floor(math.ldexp(float(v), 63 - emax))) if v > 0 else 0 for v in eps]
    tot = sum(q)
    from fractions import Fraction
    d = Fraction(float(delta))
    acc = 0
    for g, i in enumerate(sampling.error_order(eps).tolist(), start=1):
        acc += q[i]
        if acc >= d * tot:
            return min(g, npos)
    return npos


def test_fixed_point_encoding_agrees_with_exact_rule_off_the_margin():
    """The 64-bit encoding truncates each error by less than one unit of
    2^(e_max - 63), so its decision equals the exact one unless the exact
    ratio at the crossing lies within (n + N) 2^(e_max - 63) / sum(eps) of
    delta.  Indicator-like inputs never come that close; a constructed one
    does, and the difference is then the named sub-2^-64 effect."""
    rng = np.random.default_rng(5)
    for trial in range(40):
        n = int(rng.integers(20, 400))
        eps = (rng.random(n) ** 6) * 10.0 ** rng.uniform(-20, 0)
        eps[rng.random(n) < 0.1] = 0.0
        for delta in (0.3, 0.8, 0.9, 0.99, 1.0):
            assert _fixed_point_count(eps, delta) == sampling.count_g(eps, sampling.RULE_RRE, delta=delta)
    # one large error and one 2^-70 times smaller: exact RRE(1) = 1 / (1 + 2^-70) < delta
    eps = np.array([1.0, 2.0 ** -70])
    delta = 1.0 - 2.0 ** -53
    assert sampling.count_g(eps, sampling.RULE_RRE, delta=delta) == 1      # 1/(1+2^-70) > 1 - 2^-53
    eps = np.array([1.0] + [2.0 ** -60] * 256)                            # tail 2^-52 of the total
    assert sampling.count_g(eps, sampling.RULE_RRE, delta=delta) > 1
    assert _fixed_point_count(eps, delta) > 1                                # 2^-60 is still encoded
    eps = np.array([1.0] + [2.0 ** -66] * 16384)                          # tail 2^-52, each below 2^-64
    assert sampling.count_g(eps, sampling.RULE_RRE, delta=delta) > 1
    assert _fixed_point_count(eps, delta) == 1                               # the named difference


# ---------------------------------------------------------------- indicator

def test_indicator_zero_in_exact_span():
    prob, q = W.make(W.WORKLOADS["burgers2d_1024"].resized(16), 1)
    rng = np.random.default_rng(0)
    psi = q + 0.01 * rng.standard_normal(q.size)
    Phi, _ = np.linalg.qr(rng.standard_normal((q.size, 3)))
    gamma = psi + Phi @ np.array([0.3, -0.2, 0.1])
    eps, _ = sampling.indicator_full(prob, gamma, Phi, psi)
    assert np.all(eps == 0.0)
    eps2, _ = sampling.indicator_full(prob, gamma + 1e-3 * rng.standard_normal(q.size), Phi, psi)
    assert np.count_nonzero(eps2) == prob.ncell


def test_indicator_sums_components_per_cell():
    prob, q = W.make(W.WORKLOADS["euler2d_512"].resized(6), 0)
    d = np.arange(q.size, dtype=float) * 1e-3
    eps = sampling.indicator(prob, q + d, q)
    assert np.allclose(eps, (d.reshape(4, -1) ** 2).sum(axis=0), rtol=1e-12, atol=0)


# ---------------------------------------------------------------- POD

def planted(N, w, sig, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((N, w)))
    V, _ = np.linalg.qr(rng.standard_normal((w, w)))
    return U, np.asarray(sig, float), V


def test_window_mean_is_correctly_rounded():
    """The reference state is the exact mean of the window (eq. mean) with the
    sum rounded once: checked against rational arithmetic on entries with
    heavy cancellation and mixed magnitudes, where a plain left-to-right sum
    is off by many ulps."""
    from fractions import Fraction
    rng = np.random.default_rng(3)
    w, N = 7, 400
    big = rng.standard_normal(N) * 1e8
    snaps = [big, rng.standard_normal(N), -big, rng.standard_normal(N) * 1e-9, rng.standard_normal(N),
             big * 1e-8, -big * 1e-8]
    got = pod.window_mean(snaps)
    for i in range(N):
        exact = sum(Fraction(float(s_[i])) for s_ in snaps)
        want = float(exact) / w            # float(Fraction) rounds correctly; then one IEEE division
        assert got[i] == want, i
    naive = sum(snaps[1:], snaps[0]) / w
    assert np.count_nonzero(naive != got) > N // 10


def test_pod_recovers_planted_svd():
    N, w, m = 500, 6, 4
    sig = [3.0, 1.0, 0.3, 0.1, 0.03, 0.0]
    U, s, V = planted(N, w, sig, 1)
    X = U @ np.diag(s) @ V.T
    # snapshots whose deviation from the centring mean is X: use w+1 snapshots
    # g_0 = c (so the centre is c + mean of X's columns), then adjust
    base = np.random.default_rng(2).standard_normal(N)
    snaps = [base] + [base + X[:, j] for j in range(w)]
    centre, _ = pod.centring_and_new_mean(snaps, w)
    Xw = np.stack([s_ - centre for s_ in snaps[1:]], axis=1)
    out = pod.pod(snaps, w, m)
    sv = np.linalg.svd(Xw, compute_uv=False)
    assert np.allclose(out["sigma"], sv, rtol=0, atol=1e-14 * sv[0])
    Phi = out["Phi"]
    assert out["m_eff"] == m
    assert np.max(np.abs(Phi.T @ Phi - np.eye(m))) < 1e-14
    # Eckart-Young: residual energy equals the discarded singular values
    res = Xw - Phi @ (Phi.T @ Xw)
    assert abs(np.sum(res ** 2) - np.sum(sv[m:] ** 2)) < 1e-12 * np.sum(sv ** 2)


def test_pod_planted_subspace_direct():
    # centring chosen so that X itself is the planted matrix
    N, w, m = 300, 5, 3
    U, s, V = planted(N, w, [2.0, 0.7, 0.2, 0.05, 0.01], 4)
    X = U @ np.diag(s) @ V.T
    c = np.random.default_rng(5).standard_normal(N)
    # w+1 snapshots g_0..g_w with mean(g_0..g_{w-1}) = c and g_j - c = X[:, j-1] for j >= 1
    tail = [c + X[:, j] for j in range(w)]
    g0 = w * c - sum(tail[:-1])
    snaps = [g0] + tail
    out = pod.pod(snaps, w, m)
    assert np.allclose(out["sigma"], s, rtol=0, atol=1e-13 * s[0])
    P = out["Phi"] @ out["Phi"].T
    Pt = U[:, :m] @ U[:, :m].T
    assert np.max(np.abs(P - Pt)) < 1e-13


def test_pod_first_update_centres_on_own_mean_and_truncates():
    rng = np.random.default_rng(9)
    w, N = 6, 200
    snaps = [rng.standard_normal(N) for _ in range(w)]
    out = pod.pod(snaps, w, m=6)
    assert np.array_equal(out["psi_centre"], out["psi_new"])
    # centred on its own mean: rank <= w-1, the last singular value is rounding
    assert out["sigma"][-1] < 1e-13 * out["sigma"][0]
    assert out["m_eff"] == w - 1


def test_pod_sign_convention():
    rng = np.random.default_rng(1)
    snaps = [rng.standard_normal(50) for _ in range(5)]
    out = pod.pod(snaps, 4, 3)
    for i in range(out["m_eff"]):
        v = out["V"][:, i]
        assert v[np.argmax(np.abs(v))] > 0
        # left vector consistent with the right one: X v = sigma u
        assert np.allclose(out["X"] @ v, out["sigma"][i] * out["Phi"][:, i], atol=1e-13)


def test_pod_of_zero_window_is_empty():
    snaps = [np.ones(10)] * 4
    out = pod.pod(snaps, 4, 2)
    assert out["m_eff"] == 0 and out["Phi"].shape == (10, 0)


# ---------------------------------------------------------------- filter

def periodic_row(nx):
    return W.Problem(kind=W.BURGERS_2D, nx=nx, ny=1, bc=W.BC_PERIODIC, dx=1 / nx, dy=1.0,
                     dt=0.1, gamma=1.4, inflow=0.0)


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("k", [1, 3, 7, 16])
def test_shapiro_transfer_function(n, k):
    nx = 32
    prob = periodic_row(nx)
    x = np.arange(nx) / nx
    u = np.cos(2 * np.pi * k * x)
    out = hybrid.shapiro(prob, u, n)
    gain = 1.0 - np.sin(np.pi * k / nx) ** (2 * n)
    assert np.max(np.abs(out - gain * u)) < 1e-15 * 4 ** n


def test_shapiro_weights_and_invariants():
    prob = periodic_row(16)
    e = np.zeros(16)
    e[8] = 1.0
    expect = {1: [1, 2, 1], 2: [-1, 4, 10, 4, -1], 3: [1, -6, 15, 44, 15, -6, 1]}
    for n, wts in expect.items():
        out = hybrid.shapiro(prob, e, n)
        den = 4 ** n
        assert np.allclose(out[8 - n:8 + n + 1], np.array(wts) / den, atol=1e-16)
        assert np.allclose(hybrid.shapiro(prob, np.full(16, 2.5), n), 2.5, atol=1e-15)
        alt = np.cos(np.pi * np.arange(16))
        assert np.max(np.abs(hybrid.shapiro(prob, alt, n))) < 1e-14


def test_shapiro_edge_extrapolation_and_two_dimensions():
    wl = W.WORKLOADS["euler2d_512"].resized(9, 7)
    prob, _ = W.make(wl, 0)
    rng = np.random.default_rng(3)
    q = rng.standard_normal(prob.n)
    out = hybrid.shapiro(prob, q, 1).reshape(4, 7, 9)
    g = q.reshape(4, 7, 9)
    # x then y, each with the boundary value repeated outside the domain
    gp = np.pad(g, ((0, 0), (0, 0), (1, 1)), mode="edge")
    fx = (gp[:, :, :-2] + 2 * gp[:, :, 1:-1] + gp[:, :, 2:]) / 4
    fp = np.pad(fx, ((0, 0), (1, 1), (0, 0)), mode="edge")
    fy = (fp[:, :-2] + 2 * fp[:, 1:-1] + fp[:, 2:]) / 4
    assert np.max(np.abs(out - fy)) < 1e-14


def test_filter_is_identity_on_converged_hdm_state():
    prob, q0 = W.make(W.WORKLOADS["burgers2d_1024"].resized(20), 2)
    q1, _ = fv.hdm_step(prob, q0)
    out = hybrid.spatial_filter(prob, q1, q0, hybrid.HybridParams())
    assert np.array_equal(out, q1)


def filter_case_oscillation():
    """Periodic 2D Burgers, q_prev = 1 and gamma = 1 + (-1)^i / 4: the
    order-2 Shapiro filter S_1 maps the 2 dx mode to 0 and keeps constants,
    exactly in binary arithmetic for these values, and R(1; 1) = 0."""
    prob, _ = W.make(W.WORKLOADS["burgers2d_1024"].resized(32, 4), 0)
    q_prev = np.ones(prob.n)
    i = np.arange(prob.ncell) % prob.nx
    gamma = 1.0 + 0.25 * np.where(i % 2 == 0, 1.0, -1.0)
    return prob, gamma, q_prev


def filter_case_mode(amp=1e-4, k=2):
    """Periodic 2D Burgers with a step so small that R(q; 1) = q - 1 exactly,
    and gamma = 1 + amp cos(2 pi k (x_i + 1/2) / nx) (no cell on a node of the
    mode): every pass of S_n scales the mode by g_n = 1 - sin(pi k / nx)^(2n)
    (its transfer function), so every cell's residual drops by that factor
    and the relative l1 decrease of a pass is sin(pi k / nx)^(2n)."""
    import dataclasses
    prob, _ = W.make(W.WORKLOADS["burgers2d_1024"].resized(32, 4), 0)
    prob = dataclasses.replace(prob, dt=1e-300)
    q_prev = np.ones(prob.n)
    i = np.arange(prob.ncell) % prob.nx
    p = amp * np.cos(2.0 * np.pi * k * (i + 0.5) / prob.nx)
    return prob, 1.0 + p, q_prev, p, math.sin(math.pi * k / prob.nx) ** 2


def test_filter_loop_strict_gate_and_empty_stop():
    """Pass 1 of order 2 removes the oscillation in every cell; every later
    pass finds no strict decrease and ends its order at once (a non-strict
    gate would keep cells with equal zero residuals and run on)."""
    prob, gamma, q_prev = filter_case_oscillation()
    log = []
    out = hybrid.spatial_filter(prob, gamma, q_prev, hybrid.HybridParams(), log)
    assert log == [(1, 1, prob.ncell), (1, 2, 0), (2, 1, 0), (3, 1, 0)]
    assert np.array_equal(out, q_prev)


def test_filter_loop_relative_decrease_stop_and_pass_bound():
    """Order 2: the relative decrease sin^2(pi/16) = 0.038 stays above
    eps_f = 1e-2, so the order runs to j_f,max = 10 passes; orders 4 and 6
    decrease by sin^4 = 1.4e-3 and sin^6 = 5.5e-5 < eps_f and stop after one
    pass.  The amplitude makes the absolute l1 decrease (3e-4) smaller than
    eps_f, so an absolute reading of the stop test would end order 2 after
    its first pass.  The final state is 1 + g_1^10 g_2 g_3 p (one missing or
    extra pass would move it by 4e-6)."""
    prob, gamma, q_prev, p, s2 = filter_case_mode()
    assert s2 > 1e-2 and s2 * s2 < 1e-2
    assert np.sum(np.abs(p)) * s2 < 1e-2
    log = []
    out = hybrid.spatial_filter(prob, gamma, q_prev, hybrid.HybridParams(), log)
    N = prob.ncell
    assert log == [(1, j, N) for j in range(1, 11)] + [(2, 1, N), (3, 1, N)]
    gain = (1 - s2) ** 10 * (1 - s2 ** 2) * (1 - s2 ** 3)
    assert np.max(np.abs((out - 1.0) - gain * p)) <= 1e-14   # rounding of states near 1, 13 passes
    # a smaller bound ends order 2 earlier with the same per-pass factor
    log = []
    out = hybrid.spatial_filter(prob, gamma, q_prev, hybrid.HybridParams(jfmax=3), log)
    assert log == [(1, 1, N), (1, 2, N), (1, 3, N), (2, 1, N), (3, 1, N)]
    gain = (1 - s2) ** 3 * (1 - s2 ** 2) * (1 - s2 ** 3)
    assert np.max(np.abs((out - 1.0) - gain * p)) <= 1e-14   # rounding of states near 1, 13 passes


def test_filter_loop_carries_the_merged_residual_between_passes():
    """With eps_f between the order-2 and order-4 decreases only order 2
    stops early: an eps_f above 0.038 ends it after pass 1 (the decrease is
    measured against the merged state's residual, the next pass's r)."""
    prob, gamma, q_prev, p, s2 = filter_case_mode()
    N = prob.ncell
    log = []
    hybrid.spatial_filter(prob, gamma, q_prev, hybrid.HybridParams(eps_f=0.05), log)
    assert log == [(1, 1, N), (2, 1, N), (3, 1, N)]
    log = []
    hybrid.spatial_filter(prob, gamma, q_prev, hybrid.HybridParams(eps_f=1e-3), log)
    assert log == [(1, j, N) for j in range(1, 11)] + [(2, j, N) for j in range(1, 11)] + [(3, 1, N)]


# ---------------------------------------------------------------- hybrid step

@pytest.mark.parametrize("name,nx", [("burgers1d_1k", 64), ("burgers2d_1024", 14), ("euler2d_512", 10)])
def test_hybrid_with_all_cells_sampled_equals_hdm(name, nx):
    wl = W.WORKLOADS[name].resized(nx)
    prob, q0 = W.make(wl, 1)
    q1, _ = fv.hdm_step(prob, q0)
    rng = np.random.default_rng(0)
    Phi, _ = np.linalg.qr(rng.standard_normal((prob.n, 3)))
    psi = q0.copy()
    hat = np.arange(prob.ncell)
    out = hybrid.hybrid_step(prob, q0, Phi, psi, hat, np.array([], dtype=int))
    assert out["J"] == 2
    assert np.max(np.abs(out["gamma"] - q1)) <= 2 * fv.newton_tol(q0) * 10


def test_hybrid_exact_span_reproduces_hdm():
    wl = W.WORKLOADS["burgers2d_1024"].resized(16)
    prob, q0 = W.make(wl, 2)
    q1, _ = fv.hdm_step(prob, q0)
    psi = 0.5 * (q0 + q1)
    rng = np.random.default_rng(1)
    B = np.stack([q1 - psi, rng.standard_normal(prob.n), rng.standard_normal(prob.n)], axis=1)
    Phi, _ = np.linalg.qr(B)
    sel = sampling.select(prob, np.abs(q1 - q0), sampling.RULE_FRACTION, 0.1)
    params = hybrid.HybridParams(eps_y=1e-13, jmax=200)
    out = hybrid.hybrid_step(prob, q0, Phi, psi, sel["hat"], sel["tilde"], params)
    assert np.max(np.abs(out["gamma"] - q1)) < 1e-11


def test_hybrid_subiterations_at_least_two_and_bounded():
    wl = W.WORKLOADS["burgers1d_1k"].resized(128)
    prob, q0 = W.make(wl, 0)
    res = arom.run(prob, q0, 60, arom.AromParams(w=wl.w, m=wl.m, z=wl.z, fraction=wl.frac))
    Js = [r["J"] for r in res["records"] if r["type"] == "hybrid"]
    assert Js and all(2 <= j <= 10 for j in Js)


def test_unfiltered_hybrid_indicator_zero_off_sampled_set():
    wl = W.WORKLOADS["burgers2d_1024"].resized(18)
    prob, q0 = W.make(wl, 3)
    snaps = [q0]
    for _ in range(wl.w):
        snaps.append(fv.hdm_step(prob, snaps[-1])[0])
    b = pod.pod(snaps[-wl.w - 1:], wl.w, 6)
    eps, _ = sampling.indicator_full(prob, snaps[-1], b["Phi"], b["psi_new"])
    sel = sampling.select(prob, eps, sampling.RULE_FRACTION, 0.05)
    params = hybrid.HybridParams(filter_orders=())
    out = hybrid.hybrid_step(prob, snaps[-1], b["Phi"], b["psi_new"], sel["hat"], sel["tilde"], params)
    off = ~sel["mask"]
    assert np.all(out["eps"][off] == 0.0)
    d = (out["gamma"] - out["rho"])[sel["hat"]]
    assert np.allclose(out["eps"][sel["hat"]], np.where(d * d < (sampling.DEFAULT_FLOOR * max(1.0, np.max(np.abs(out["gamma"])))) ** 2, 0, d * d))


# ---------------------------------------------------------------- Algorithm 1 schedule

def test_schedule_closed_form_burgers1d():
    wl = W.WORKLOADS["burgers1d_1k"]
    prob, q0 = W.make(wl, 0)
    res = arom.run(prob, q0, wl.steps, arom.AromParams(w=wl.w, m=wl.m, z=wl.z, fraction=wl.frac))
    full = [r["k"] for r in res["records"] if r["type"] == "full"]
    expect = list(range(1, wl.w + 1)) + list(range(20, wl.steps + 1, 20))
    assert full == expect and len(full) == 25
    updates = [r["k"] for r in res["records"] if "m_eff" in r]
    assert updates == [k for k in range(wl.w - 1, wl.steps) if (k + 1) % wl.z != 0]
