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


def test_rre_fixed_point_encoding():
    eps = np.array([0.0, 3.0, 1.5, 2.0 ** -70, 1.0])
    q = sampling.fixed_point_errors(eps)
    # largest 3 = 1.5 * 2^1 -> 3 * 2^62; others scale alike; 2^-70 * 2^62 < 1 -> 0
    assert q == [0, 3 << 62, 3 << 61, 0, 1 << 62]


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
    assert np.allclose(out["eps"][sel["hat"]], np.where(d * d < (1e-11 * np.max(np.abs(out["gamma"]))) ** 2, 0, d * d))


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
