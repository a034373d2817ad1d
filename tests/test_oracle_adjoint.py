"""Pins of the oracle adjoint (no GPU): transposes by the dot-product test,
the tangent/adjoint pair of each step type, replay of the taped trajectory,
and central finite differences of the frozen-decision trajectory map."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as A
from oracle import fv
from oracle.arom import AromParams
from oracle.hybrid import HybridParams, shapiro


@pytest.mark.parametrize("name,nx,ny", [("burgers1d_1k", 37, 1), ("burgers2d_1024", 13, 11),
                                        ("euler2d_512", 9, 7)])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_shapiro_transpose_dot_product(name, nx, ny, n):
    prob, _ = W.make(W.WORKLOADS[name].resized(nx, ny), 0)
    rng = np.random.default_rng(n)
    u = rng.standard_normal(prob.n)
    v = rng.standard_normal(prob.n)
    lhs = shapiro(prob, u, n) @ v
    rhs = u @ A.shapiro_T(prob, v, n)
    assert abs(lhs - rhs) <= 1e-14 * max(abs(lhs), 1.0) * prob.n ** 0.5


def small_case(name, nx, ny, m, seed, fraction=0.08):
    wl = W.WORKLOADS[name].resized(nx, ny, m=m)
    prob, q0 = W.make(wl, seed)
    p = AromParams(w=wl.w, m=wl.m, z=wl.z, fraction=fraction, halo=1)
    return wl, prob, q0, p


# On 96 cells a fraction of 8 % leaves about 11 fit rows for 6 modes; such
# nearly square gathered bases reach condition numbers near 1e5, whose
# kappa^2 eps rounding noise in the fit swamps a central difference at
# h = 1e-6.  15 % keeps kappa below 200 (measured).
CASES = {"burgers2d": ("burgers2d_1024", 18, 16, 6, 3), "euler2d": ("euler2d_512", 12, 10, 4, 1),
         "burgers1d": ("burgers1d_1k", 96, 1, 6, 2, 0.15)}


@pytest.fixture(scope="module", params=list(CASES))
def taped(request):
    wl, prob, q0, p = small_case(*CASES[request.param])
    steps = wl.w + 8
    qT, tape = A.forward_with_tape(prob, q0, steps, p)
    return wl, prob, q0, p, qT, tape


def test_tape_has_both_step_types(taped):
    *_, tape = taped
    kinds = [st["type"] for st in tape]
    assert "hybrid" in kinds and "full" in kinds


def test_replay_reproduces_forward(taped):
    wl, prob, q0, p, qT, tape = taped
    qr = A.replay(prob, q0, tape, p.hybrid)
    assert np.linalg.norm(qr - qT) <= 1e-12 * np.linalg.norm(qT)


@pytest.mark.parametrize("kind", ["full", "hybrid"])
def test_step_tangent_adjoint_dot_product(taped, kind):
    wl, prob, q0, p, qT, tape = taped
    st = next(s for s in tape if s["type"] == kind)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(prob.n)
    w = rng.standard_normal(prob.n)
    Tv = A.step_tangent(prob, st, v, p.hybrid)
    Ttw = A.step_adjoint(prob, st, w, p.hybrid)
    lhs, rhs = Tv @ w, v @ Ttw
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.linalg.norm(Tv) * np.linalg.norm(w))


def test_hybrid_tangent_matches_finite_difference(taped):
    wl, prob, q0, p, qT, tape = taped
    k = next(i for i, s in enumerate(tape) if s["type"] == "hybrid")
    st = tape[k]
    q_prev = A.replay(prob, q0, tape[:k], p.hybrid)
    d = np.random.default_rng(2).standard_normal(prob.n)
    h = 1e-6
    fd = (A.replay_hybrid(prob, q_prev + h * d, st, p.hybrid)
          - A.replay_hybrid(prob, q_prev - h * d, st, p.hybrid)) / (2 * h)
    t = A.step_tangent(prob, st, d, p.hybrid)
    assert np.linalg.norm(fd - t) <= 1e-6 * np.linalg.norm(t)


def test_trajectory_gradient_central_differences(taped):
    wl, prob, q0, p, qT, tape = taped
    target = fv.hdm_step(prob, q0 * 1.01)[0]
    g = A.gradient(prob, tape, qT, target, p.hybrid)
    rng = np.random.default_rng(11)
    h = 1e-6
    for _ in range(16):
        d = rng.standard_normal(prob.n)
        Lp = A.loss(A.replay(prob, q0 + h * d, tape, p.hybrid), target)
        Lm = A.loss(A.replay(prob, q0 - h * d, tape, p.hybrid), target)
        fd = (Lp - Lm) / (2 * h)
        gd = g @ d
        assert abs(gd - fd) <= 1e-6 * max(abs(gd), 1e-8 * np.linalg.norm(g) * np.linalg.norm(d)), (gd, fd)


# ---------------------------------------------------------------- through psi
def test_hybrid_psi_adjoint_dot_product(taped):
    """The psi-adjoint of a hybrid step is the transpose of its psi-tangent,
    and its gamma_{k-1} part equals the frozen-psi adjoint bit for bit."""
    wl, prob, q0, p, qT, tape = taped
    st = next(s for s in tape if s["type"] == "hybrid")
    rng = np.random.default_rng(5)
    dpsi = rng.standard_normal(prob.n)
    w = rng.standard_normal(prob.n)
    Td = A.hybrid_step_tangent_psi(prob, st, dpsi, p.hybrid)
    pbar, psibar = A.hybrid_step_adjoint_psi(prob, st, w, p.hybrid)
    lhs, rhs = Td @ w, dpsi @ psibar
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.linalg.norm(Td) * np.linalg.norm(w))
    assert np.array_equal(pbar, A.hybrid_step_adjoint(prob, st, w, p.hybrid))


def test_hybrid_psi_tangent_matches_finite_difference(taped):
    wl, prob, q0, p, qT, tape = taped
    k = next(i for i, s in enumerate(tape) if s["type"] == "hybrid")
    st = tape[k]
    q_prev = A.replay(prob, q0, tape[:k], p.hybrid)
    d = np.random.default_rng(3).standard_normal(prob.n)
    h = 1e-6
    fd = (A.replay_hybrid(prob, q_prev, dict(st, psi=st["psi"] + h * d), p.hybrid)
          - A.replay_hybrid(prob, q_prev, dict(st, psi=st["psi"] - h * d), p.hybrid)) / (2 * h)
    t = A.hybrid_step_tangent_psi(prob, st, d, p.hybrid)
    assert np.linalg.norm(fd - t) <= 1e-6 * np.linalg.norm(t)


def test_psi_indices_are_the_means_snapshots(taped):
    """Each hybrid step's psi is the plain mean of the snapshots it lists
    (the last w of its basis update's window, eq. mean)."""
    wl, prob, q0, p, qT, tape = taped
    states = [q0]
    for st in tape:
        states.append(st["out"])
    for st in tape:
        if st["type"] != "hybrid":
            continue
        idx = st["psi_idx"]
        assert len(idx) == wl.w and idx == list(range(idx[0], idx[0] + wl.w))
        mean = sum(states[j] for j in idx) / wl.w
        assert np.max(np.abs(mean - st["psi"])) <= 1e-14 * np.max(np.abs(mean))


def test_trajectory_gradient_through_psi_central_differences(taped):
    """With psi_live the gradient is that of the trajectory whose reference
    states are recomputed from the perturbed run (bases and decisions
    frozen); the psi path is not negligible: the frozen-psi gradient misses
    these differences."""
    wl, prob, q0, p, qT, tape = taped
    target = fv.hdm_step(prob, q0 * 1.01)[0]
    g = A.gradient(prob, tape, qT, target, p.hybrid, psi_live=True)
    g0 = A.gradient(prob, tape, qT, target, p.hybrid)
    assert np.linalg.norm(g - g0) > 1e-4 * np.linalg.norm(g)
    rng = np.random.default_rng(13)
    h = 1e-6
    for _ in range(16):
        d = rng.standard_normal(prob.n)
        Lp = A.loss(A.replay(prob, q0 + h * d, tape, p.hybrid, psi_live=True), target)
        Lm = A.loss(A.replay(prob, q0 - h * d, tape, p.hybrid, psi_live=True), target)
        fd = (Lp - Lm) / (2 * h)
        gd = g @ d
        assert abs(gd - fd) <= 1e-6 * max(abs(gd), 1e-8 * np.linalg.norm(g) * np.linalg.norm(d)), (gd, fd)
