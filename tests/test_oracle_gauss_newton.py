"""Pins of the oracle's full-sensitivity Gauss-Newton subiterations (no GPU):
the gradient A^T r against central differences of the misfit with the
partial solve redone (validates dv/dy = -J_S^-1 J_T Phi_T), stationarity at
the Gauss-Newton point against the paper's fixed point, quadratic decay of
the steps near a zero-residual solution, a single step when nothing is held
(all cells sampled), and recovery of a state in the affine subspace."""
import numpy as np
import pytest

import workloads as W
from oracle import fv, gauss_newton as gn, hybrid, pod, sampling


def setup(name, nx, seed, w=8, m=5, frac=0.1):
    wl = W.WORKLOADS[name].resized(nx)
    prob, q0 = W.make(wl, seed)
    snaps = [q0]
    for _ in range(w):
        snaps.append(fv.hdm_step(prob, snaps[-1])[0])
    b = pod.pod(snaps[-w - 1:], w, m)
    eps, _ = sampling.indicator_full(prob, snaps[-1], b["Phi"], b["psi_new"])
    sel = sampling.select(prob, eps, sampling.RULE_FRACTION, frac, halo=1)
    return prob, snaps[-1], b["Phi"], b["psi_new"], sel


def misfit(prob, q_prev, Phi, psi, sel, y):
    hd = fv.dofs_of_cells(prob, sel["hat"])
    td = fv.dofs_of_cells(prob, sel["tilde"])
    u = q_prev.copy()
    u[td] = psi[td] + Phi[td] @ y
    u, _ = fv.partial_hdm_solve(prob, u, q_prev, sel["hat"], tol=1e-15)
    r = Phi[hd] @ y - (u[hd] - psi[hd])
    return 0.5 * float(r @ r), r, u


@pytest.mark.parametrize("name,nx,seed", [("burgers1d_1k", 200, 0), ("burgers2d_1024", 22, 1), ("euler2d_512", 14, 2)])
def test_gradient_matches_central_differences(name, nx, seed):
    prob, q, Phi, psi, sel = setup(name, nx, seed)
    hd = fv.dofs_of_cells(prob, sel["hat"])
    td = fv.dofs_of_cells(prob, sel["tilde"])
    y = np.linalg.lstsq(Phi[hd], q[hd] - psi[hd], rcond=None)[0]
    f, r, u = misfit(prob, q, Phi, psi, sel, y)
    A, _ = gn.residual_jacobian(prob, u, q, hd, td, Phi)
    g = A.T @ r
    rng = np.random.default_rng(seed)
    h = 1e-6 * max(1.0, float(np.linalg.norm(y)))
    for _ in range(4):
        d = rng.standard_normal(y.size)
        d /= np.linalg.norm(d)
        fd = (misfit(prob, q, Phi, psi, sel, y + h * d)[0] - misfit(prob, q, Phi, psi, sel, y - h * d)[0]) / (2 * h)
        assert abs(g @ d - fd) <= 1e-6 * max(abs(fd), 1e-8 * np.linalg.norm(g)), (g @ d, fd)


@pytest.mark.parametrize("name,nx,seed", [("burgers1d_1k", 200, 0), ("burgers2d_1024", 22, 1)])
def test_gauss_newton_point_is_stationary_and_differs_from_the_paper_fixed_point(name, nx, seed):
    prob, q, Phi, psi, sel = setup(name, nx, seed)
    params = hybrid.HybridParams(eps_y=1e-12, jmax=40)
    rec = []
    out = gn.gn_hybrid_step(prob, q, Phi, psi, sel["hat"], sel["tilde"], params, record=rec)
    hd = fv.dofs_of_cells(prob, sel["hat"])
    td = fv.dofs_of_cells(prob, sel["tilde"])
    f, r, u = misfit(prob, q, Phi, psi, sel, out["y"])
    A, X = gn.residual_jacobian(prob, u, q, hd, td, Phi)
    assert np.linalg.norm(A.T @ r) <= 1e-9 * np.linalg.norm(A) * max(np.linalg.norm(r), 1e-12)
    # the paper's subiterations converge to Phi_S^T r = 0 instead, where A^T r != 0
    ref = hybrid.hybrid_step(prob, q, Phi, psi, sel["hat"], sel["tilde"], hybrid.HybridParams(eps_y=1e-12, jmax=200))
    fp, rp, up = misfit(prob, q, Phi, psi, sel, ref["y"])
    assert np.linalg.norm(Phi[hd].T @ rp) <= 1e-8 * np.linalg.norm(rp)
    if np.linalg.norm(X) > 1e-8:
        assert f <= fp * (1 + 1e-12)


def test_quadratic_steps_near_a_zero_residual_solution():
    """The HDM step's deviation in the span of Phi: the misfit vanishes at the
    solution, so Gauss-Newton converges quadratically."""
    wl = W.WORKLOADS["burgers2d_1024"].resized(16)
    prob, q0 = W.make(wl, 2)
    q1, _ = fv.hdm_step(prob, q0, tol=1e-15)
    psi = 0.5 * (q0 + q1)
    rng = np.random.default_rng(1)
    Phi, _ = np.linalg.qr(np.stack([q1 - psi, rng.standard_normal(prob.n), rng.standard_normal(prob.n)], axis=1))
    sel = sampling.select(prob, np.abs(q1 - q0), sampling.RULE_FRACTION, 0.1)
    params = hybrid.HybridParams(eps_y=1e-13, jmax=30, filter_orders=())
    out = gn.gn_hybrid_step(prob, q0, Phi, psi, sel["hat"], sel["tilde"], params)
    dy = out["dy"]
    assert np.max(np.abs(out["gamma"] - q1)) < 1e-11
    big = [d for d in dy if d > 1e-10]
    assert all(b <= 10 * a * a + 1e-12 for a, b in zip(big, big[1:])), dy
    # the paper's frozen iteration is only linear on the same inputs
    ref = hybrid.hybrid_step(prob, q0, Phi, psi, sel["hat"], sel["tilde"], hybrid.HybridParams(eps_y=1e-13, jmax=200,
                                                                                                 filter_orders=()))
    assert out["J"] < ref["J"]


def test_all_cells_sampled_is_one_least_squares_step():
    wl = W.WORKLOADS["burgers1d_1k"].resized(64)
    prob, q0 = W.make(wl, 1)
    q1, _ = fv.hdm_step(prob, q0)
    rng = np.random.default_rng(0)
    Phi, _ = np.linalg.qr(rng.standard_normal((prob.n, 3)))
    out = gn.gn_hybrid_step(prob, q0, Phi, q0.copy(), np.arange(prob.ncell), np.array([], dtype=int))
    assert out["J"] == 2 and out["dy"][0] < 1e-12
    assert np.max(np.abs(out["gamma"] - q1)) <= 20 * fv.newton_tol(q0)
