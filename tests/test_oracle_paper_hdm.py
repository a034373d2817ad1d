"""Pins of the oracle's version of the paper's HDM (Sec. 3.1: MUSCL with the
minmod limiter, Roe's flux, BDF2) against facts the mathematics fixes (no
GPU): Roe's eigen-decomposition and Roe property, its exact capture of a
stationary shock, consistency and upwinding, exactness of the reconstruction
on linear data, conservation with boundary fluxes, mirror and transpose
symmetries, second order in time and space, the colour-grouped Jacobian
against column-by-column differences, and convergence to the exact Riemann
solution of Sod's shock tube (Sec. 3.2)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import fv
from oracle import paper_hdm as ph
from test_oracle_fv import euler, exact_riemann, prim_to_cons

HERE = os.path.dirname(__file__)
G = 1.4


def random_states(rng, n, mach=0.8):
    rho = 0.5 + rng.random(n)
    p = 0.3 + rng.random(n)
    c = np.sqrt(G * p / rho)
    u = mach * c * (2 * rng.random(n) - 1)
    v = mach * c * (2 * rng.random(n) - 1)
    return ph.conservative(np.stack([rho, u, v, p]), G)


def fixed_problem(w, dt, nx, ny=1, bc=ph.FIXED):
    """A problem whose ghosts hold the boundary cells' initial states."""
    if ny == 1:
        ghost = (ph.conservative(w[:, :1], G)[:, 0], ph.conservative(w[:, -1:], G)[:, 0])
    else:
        ghost = ()
    return ph.PaperProblem(nx=nx, ny=ny, dx=1.0 / nx, dy=1.0 / ny, dt=dt, gamma=G, bc=bc, ghost=ghost)


# ------------------------------------------------------------------ limiter

def test_minmod_textbook_cases():
    a = np.array([1.0, -1.0, 1.0, 0.0, 2.0, -3.0, 0.5])
    b = np.array([2.0, -3.0, -1.0, 5.0, 0.0, -0.25, 0.5])
    assert np.array_equal(ph.minmod(a, b), [1.0, -1.0, 0.0, 0.0, 0.0, -0.25, 0.5])


# -------------------------------------------------------------------- Roe

@pytest.mark.parametrize("axis", [0, 1])
def test_roe_waves_decompose_the_jump_and_satisfy_roe_property(axis):
    """sum alpha_k r_k = qR - qL and sum lambda_k alpha_k r_k = F(qR) - F(qL):
    the Roe matrix's decomposition (any mistake in an eigenvector, a wave
    strength or the Roe averages breaks one of the two)."""
    rng = np.random.default_rng(11 + axis)
    qL, qR = random_states(rng, 50), random_states(rng, 50)
    lam, alpha, r = ph.roe_waves(qL, qR, G, axis)
    jump = sum(alpha[k] * r[k] for k in range(4))
    dflux = sum(lam[k] * alpha[k] * r[k] for k in range(4))
    assert np.max(np.abs(jump - (qR - qL))) < 1e-13
    dF = ph.physical_flux(qR, G, axis) - ph.physical_flux(qL, G, axis)
    assert np.max(np.abs(dflux - dF)) < 1e-13


@pytest.mark.parametrize("axis", [0, 1])
def test_roe_flux_is_consistent(axis):
    q = random_states(np.random.default_rng(3), 40)
    assert np.max(np.abs(ph.roe_flux(q, q, G, axis) - ph.physical_flux(q, G, axis))) < 1e-15


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_roe_flux_upwinds_supersonic_flow(sign):
    rng = np.random.default_rng(7)
    rho, p = 0.5 + rng.random((2, 20)), 0.5 + rng.random((2, 20))
    c = np.sqrt(G * p / rho)
    u = sign * 1.5 * c.max(axis=0) * (1 + rng.random(20))   # |u| > c on both sides
    qL = ph.conservative(np.stack([rho[0], u, 0.1 * u, p[0]]), G)
    qR = ph.conservative(np.stack([rho[1], u, -0.1 * u, p[1]]), G)
    up = qL if sign > 0 else qR
    assert np.max(np.abs(ph.roe_flux(qL, qR, G, 0) - ph.physical_flux(up, G, 0))) < 1e-13


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("mach", [1.2, 2.0, 4.0])
def test_roe_flux_captures_stationary_shock_exactly(axis, mach):
    """States joined by a stationary normal shock (textbook Rankine-Hugoniot
    relations in the upstream Mach number): Roe's flux equals the physical flux
    of either side."""
    rho1, p1 = 1.0, 1.0
    u1 = mach * math.sqrt(G * p1 / rho1)
    rho2 = rho1 * (G + 1) * mach ** 2 / ((G - 1) * mach ** 2 + 2)
    p2 = p1 * (1 + 2 * G / (G + 1) * (mach ** 2 - 1))
    u2 = u1 * rho1 / rho2
    t = 0.3                                              # tangential velocity, continuous
    w1 = [rho1, u1, t, p1] if axis == 0 else [rho1, t, u1, p1]
    w2 = [rho2, u2, t, p2] if axis == 0 else [rho2, t, u2, p2]
    q1 = ph.conservative(np.array(w1)[:, None], G)
    q2 = ph.conservative(np.array(w2)[:, None], G)
    F1, F2 = ph.physical_flux(q1, G, axis), ph.physical_flux(q2, G, axis)
    assert np.max(np.abs(F1 - F2)) < 1e-12                # the relations themselves
    assert np.max(np.abs(ph.roe_flux(q1, q2, G, axis) - F1)) < 1e-12


# ----------------------------------------------------------------- MUSCL

def test_muscl_is_exact_on_linear_data():
    """Primitive fields linear in x: both reconstructed face states equal the
    field at the face, so every interior face flux is the physical flux there
    (a left/right or half-slope mistake breaks it)."""
    nx = 20
    xc = (np.arange(nx) + 0.5) / nx
    w = np.stack([1.0 + 0.3 * xc, 0.2 - 0.1 * xc, 0.05 + 0.2 * xc, 1.0 - 0.4 * xc])
    prob = fixed_problem(w, 1e-3, nx)
    F = ph.face_fluxes(prob, ph.conservative(w, G).reshape(-1), 0)[:, 0, :]
    xf = np.arange(nx + 1) / nx
    wf = np.stack([1.0 + 0.3 * xf, 0.2 - 0.1 * xf, 0.05 + 0.2 * xf, 1.0 - 0.4 * xf])
    exact = ph.physical_flux(ph.conservative(wf, G), G, 0)
    # faces 2..nx-2 have two real cells on each side
    assert np.max(np.abs(F[:, 2:nx - 1] - exact[:, 2:nx - 1])) < 1e-14


def test_muscl_is_first_order_at_an_extremum():
    nx = 9
    rho = np.array([1.0, 1.1, 1.2, 1.3, 1.5, 1.35, 1.2, 1.1, 1.0])
    w = np.stack([rho, 0 * rho, 0 * rho, 1 + 0 * rho])
    prob = fixed_problem(w, 1e-3, nx)
    F = ph.face_fluxes(prob, ph.conservative(w, G).reshape(-1), 0)[:, 0, :]
    # faces either side of cell 4 (the maximum): that cell's face state is its
    # own value (slope 0), the neighbour's is reconstructed
    left = np.array([[1.3 + 0.5 * 0.1], [0], [0], [1]])
    right = np.array([[1.35 - 0.5 * 0.15], [0], [0], [1]])
    mid = np.array([[1.5], [0], [0], [1]])
    fl = ph.roe_flux(ph.conservative(left, G), ph.conservative(mid, G), G, 0)[:, 0]
    fr = ph.roe_flux(ph.conservative(mid, G), ph.conservative(right, G), G, 0)[:, 0]
    assert np.max(np.abs(F[:, 4] - fl)) < 1e-15 and np.max(np.abs(F[:, 5] - fr)) < 1e-15


# ------------------------------------------------------------- time steps

@pytest.mark.parametrize("ny", [1, 6])
def test_constant_state_is_fixed_point(ny):
    nx = 10
    w = np.tile(np.array([0.8, 0.3, -0.2, 1.3])[:, None], (1, nx * ny))
    q = ph.conservative(w, G).reshape(-1)
    if ny == 1:
        prob = fixed_problem(w, 0.01, nx)
    else:
        gs = tuple(ph.conservative(w[:, :1], G)[:, 0] for _ in range(4))
        prob = ph.PaperProblem(nx=nx, ny=ny, dx=0.1, dy=1 / ny, dt=0.01, gamma=G, bc=ph.FIXED, ghost=gs)
    assert np.max(np.abs(ph.rhs(prob, q))) < 1e-14
    qn, it = ph.hdm_step(prob, q, q)
    assert it == 0 and np.array_equal(qn, q)


def test_sod_balance_with_boundary_fluxes():
    """Sod's tube while the waves are inside: the boundary faces see the
    initial states, whose Roe fluxes are (0, P, 0, 0).  So mass and energy
    are conserved and the BDF combination of the total momentum equals
    beta dt (P_left - P_right) / dx per step (BDF1 on the first)."""
    nx, steps = 60, 12
    prob, q0 = ph.sod(nx, steps, T=0.05)
    states = ph.run(prob, q0, steps)
    a0, a1, a2, beta = ph.BDF2
    sums = [s.reshape(4, -1).sum(axis=1) for s in states]
    tol = 60 * nx * 1e-12
    for k in range(1, steps + 1):
        assert abs(sums[k][0] - sums[0][0]) < tol and abs(sums[k][3] - sums[0][3]) < tol
        push = prob.dt * (1.0 - 0.1) / prob.dx
        if k == 1:
            assert abs(sums[1][1] - sums[0][1] - push) < tol
        else:
            bal = a2 * sums[k][1] + a1 * sums[k - 1][1] + a0 * sums[k - 2][1]
            assert abs(bal - beta * push) < tol
        assert np.max(np.abs(states[k].reshape(4, -1)[2])) < tol          # no transverse momentum


def test_wall_conserves_mass_and_energy_2d():
    nx = ny = 8
    rng = np.random.default_rng(2)
    w = np.stack([0.8 + 0.4 * rng.random(nx * ny), 0.3 * rng.standard_normal(nx * ny),
                  0.3 * rng.standard_normal(nx * ny), 0.8 + 0.4 * rng.random(nx * ny)])
    prob = ph.PaperProblem(nx=nx, ny=ny, dx=1 / nx, dy=1 / ny, dt=0.01, gamma=G, bc=ph.WALL)
    q0 = ph.conservative(w, G).reshape(-1)
    f = ph.rhs(prob, q0).reshape(4, -1).sum(axis=1)
    assert abs(f[0]) < 1e-12 and abs(f[3]) < 1e-12
    q1, _ = ph.hdm_step(prob, q0)
    q2, _ = ph.hdm_step(prob, q1, q0)
    for q in (q1, q2):
        d = (q - q0).reshape(4, -1).sum(axis=1)
        assert abs(d[0]) < 1e-10 and abs(d[3]) < 1e-10


def test_mirror_symmetry_1d():
    """x -> 1 - x (cells reversed, u negated, ghosts swapped) commutes with a
    BDF2 step."""
    nx = 24
    rng = np.random.default_rng(9)
    w = np.stack([0.8 + 0.4 * rng.random(nx), 0.3 * rng.standard_normal(nx), 0 * np.ones(nx),
                  0.8 + 0.4 * rng.random(nx)])
    q0 = ph.conservative(w, G).reshape(-1)

    def mirror(q):
        m = q.reshape(4, -1)[:, ::-1].copy()
        m[1] *= -1
        return m.reshape(-1)

    prob = fixed_problem(w, 0.005, nx)
    wm = ph.primitive(mirror(q0).reshape(4, -1), G)
    probm = fixed_problem(wm, 0.005, nx)
    q1, _ = ph.hdm_step(prob, q0)
    q2, _ = ph.hdm_step(prob, q1, q0)
    m1, _ = ph.hdm_step(probm, mirror(q0))
    m2, _ = ph.hdm_step(probm, m1, mirror(q0))
    assert np.max(np.abs(mirror(q2) - m2)) < 1e-11


def test_2d_y_uniform_equals_1d_and_transpose_symmetry():
    nx = ny = 10
    rng = np.random.default_rng(4)
    w1 = np.stack([0.8 + 0.4 * rng.random(nx), 0.3 * rng.standard_normal(nx), 0 * np.ones(nx),
                   0.8 + 0.4 * rng.random(nx)])
    p1 = ph.PaperProblem(nx=nx, ny=1, dx=1 / nx, dy=1.0, dt=0.01, gamma=G, bc=ph.WALL)
    p2 = ph.PaperProblem(nx=nx, ny=ny, dx=1 / nx, dy=1 / ny, dt=0.01, gamma=G, bc=ph.WALL)
    q1 = ph.conservative(w1, G)
    q2 = np.repeat(q1[:, None, :], ny, axis=1)
    f1 = ph.rhs(p1, q1.reshape(-1)).reshape(4, 1, nx)
    f2 = ph.rhs(p2, q2.reshape(-1)).reshape(4, ny, nx)
    assert np.max(np.abs(f2 - f1)) < 1e-13
    # transpose: q(x, y) -> q(y, x) with the velocity components swapped
    w = np.stack([0.8 + 0.4 * rng.random((ny, nx)), 0.3 * rng.standard_normal((ny, nx)),
                  0.3 * rng.standard_normal((ny, nx)), 0.8 + 0.4 * rng.random((ny, nx))])
    q = ph.conservative(w, G)
    qt = q.transpose(0, 2, 1)[[0, 2, 1, 3]]
    f = ph.rhs(p2, q.reshape(-1)).reshape(4, ny, nx)
    ft = ph.rhs(p2, qt.copy().reshape(-1)).reshape(4, ny, nx)
    assert np.max(np.abs(ft - f.transpose(0, 2, 1)[[0, 2, 1, 3]])) < 1e-13


def _entropy_wave(nx, steps, T=0.1):
    """A monotone density front carried at u = 0.5 (constant pressure): the
    exact solution is the translated profile."""
    x = (np.arange(nx) + 0.5) / nx
    prof = lambda s: 1 + 0.2 * np.tanh((s - 0.4) / 0.08)
    w = np.stack([prof(x), 0.5 + 0 * x, 0 * x, 1 + 0 * x])
    prob = fixed_problem(w, T / steps, nx)
    return prob, ph.conservative(w, G).reshape(-1), prof(x - 0.5 * T)


def test_bdf2_is_second_order_in_time():
    """Fixed mesh, dt halved: the error against a fine-step solution falls
    by four (a wrong BDF coefficient makes the scheme inconsistent or first
    order)."""
    prob, q0, _ = _entropy_wave(64, 10)
    run = lambda steps: ph.run(ph.PaperProblem(**{**prob.__dict__, "dt": 0.1 / steps}), q0, steps)[-1]
    ref = run(320)
    errs = [np.max(np.abs(run(s) - ref)) for s in (20, 40, 80)]
    assert all(errs[i] / errs[i + 1] > 3.5 for i in range(2)), errs


def test_muscl_is_second_order_on_monotone_data():
    errs = []
    for nx in (50, 100, 200):
        prob, q0, exact = _entropy_wave(nx, nx // 2)
        q = ph.run(prob, q0, nx // 2)[-1]
        errs.append(np.mean(np.abs(q[:nx] - exact)))
    assert all(errs[i] / errs[i + 1] > 3.0 for i in range(2)), errs


# --------------------------------------------------------------- Jacobian

@pytest.mark.parametrize("nx,ny,bc", [(13, 1, ph.FIXED), (7, 6, ph.WALL)])
def test_coloured_jacobian_equals_column_by_column(nx, ny, bc):
    rng = np.random.default_rng(1)
    n = nx * ny
    w = np.stack([0.8 + 0.4 * rng.random(n), 0.3 * rng.standard_normal(n), 0.3 * rng.standard_normal(n),
                  0.8 + 0.4 * rng.random(n)])
    if ny == 1:
        w[2] = 0.0
    prob = fixed_problem(w, 0.01, nx, ny, bc) if bc == ph.FIXED else \
        ph.PaperProblem(nx=nx, ny=ny, dx=1 / nx, dy=1 / ny, dt=0.01, gamma=G, bc=bc)
    q = ph.conservative(w, G).reshape(-1)
    q1 = q * (1 + 0.01 * rng.standard_normal(q.size))
    J = ph.fd_jacobian(prob, q, q1, q1).toarray()
    R0 = ph.residual(prob, q, q1, q1)
    for col in range(q.size):
        h = 1e-7 * max(1.0, abs(q[col]))
        qp = q.copy()
        qp[col] += h
        assert np.array_equal(J[:, col], (ph.residual(prob, qp, q1, q1) - R0) / h), col


# ------------------------------------------------------------------- Sod

def test_sod_converges_to_exact_riemann_solution_and_beats_first_order():
    """Sec. 3.2's problem: the L1 density error against the exact Riemann
    solution falls with the mesh, and is well below that of the first-order
    Rusanov / backward-Euler scheme on the same mesh and steps."""
    sod = json.load(open(os.path.join(HERE, "golden", "paper_parameters.json")))["sod"]
    errs = []
    for nx in (100, 200):
        prob, q0 = ph.sod(nx, nx, T=sod["T"], gamma=G)
        q = ph.run(prob, q0, nx)[-1]
        x = (np.arange(nx) + 0.5) / nx
        re, ue, pe, *_ = exact_riemann(sod["left"], sod["right"], G, (x - sod["x0"]) / sod["T"])
        w = ph.primitive(q.reshape(4, -1), G)
        errs.append(np.mean(np.abs(w[0] - re)))
        if nx == 100:
            assert np.mean(np.abs(w[1] - ue)) < 0.02 and np.mean(np.abs(w[3] - pe)) < 0.01
            q1 = prim_to_cons(np.where(x < 0.5, 1.0, 0.125), 0 * x, 0 * x, np.where(x < 0.5, 1.0, 0.1))
            p1 = euler(nx, 1, prob.dt)
            for _ in range(nx):
                q1, _ = fv.hdm_step(p1, q1)
            e1 = np.mean(np.abs(q1[:nx] - re))
            assert errs[0] < 0.6 * e1, (errs[0], e1)
    assert errs[0] < 0.01 and errs[0] / errs[1] > 1.6, errs


# ------------------------------------------- Alg. 1 with the paper's HDM

from oracle import arom, paper_arom as pa, pod, sampling  # noqa: E402


def _sod_states(nx, steps, k):
    prob, q0 = ph.sod(nx, steps)
    return prob, ph.run(prob, q0, k, rtol=1e-13)


@pytest.mark.parametrize("nx,ny", [(17, 1), (9, 8)])
def test_ring_holds_everything_the_sampled_residual_reads(nx, ny):
    """Brute force: replacing every cell outside the sampled set and its ring
    by another state leaves the sampled cells' residual bit for bit the same,
    and every cell on which that residual depends numerically (a non-zero
    column of the Jacobian's sampled rows) lies in the ring."""
    rng = np.random.default_rng(nx)
    n = nx * ny

    def state():
        w = np.stack([0.8 + 0.4 * rng.random(n), 0.3 * rng.standard_normal(n), 0.3 * rng.standard_normal(n),
                      0.8 + 0.4 * rng.random(n)])
        if ny == 1:
            w[2] = 0.0
        return ph.conservative(w, G).reshape(-1)

    prob = ph.PaperProblem(nx=nx, ny=ny, dx=1 / nx, dy=1 / ny, dt=0.01, gamma=G, bc=ph.WALL)
    q, q1, other = state(), state(), state()
    J = ph.fd_jacobian(prob, q, q1, q1).toarray()
    for trial in range(6):
        mask = rng.random(n) < 0.2
        rg = pa.ring(prob, mask)
        rows = pa.dofs(prob, np.flatnonzero(mask))
        far = pa.dofs(prob, np.flatnonzero(~mask & ~rg))
        qf = q.copy()
        qf[far] = other[far]
        assert np.array_equal(ph.residual(prob, qf, q1, q1)[rows], ph.residual(prob, q, q1, q1)[rows]), trial
        touched = np.any(J[rows] != 0.0, axis=0).reshape(4, n).any(axis=0)
        assert not np.any(touched & ~mask & ~rg), trial


def test_paper_hybrid_all_sampled_equals_hdm_step():
    prob, states = _sod_states(60, 120, 12)
    q1, q2 = states[-1], states[-2]
    snaps = states[-6:-1]
    b = pod.pod(snaps, 5, 4)
    out = pa.hybrid_step(prob, q1, q2, b["Phi"], b["psi_new"], np.arange(prob.ncell))
    q, _ = ph.hdm_step(prob, q1, q2, rtol=1e-13)
    assert out["l"] == 0 and out["J"] == 2
    assert np.max(np.abs(out["gamma"] - q)) < 1e-11


def test_paper_hybrid_recovers_a_state_in_the_affine_subspace():
    """psi = gamma_{k-1} and Phi the direction to the HDM's gamma_k: the
    subiterations converge to gamma_k (the fixed point is the exact state),
    which the filters keep."""
    prob, states = _sod_states(80, 160, 20)
    q1, q2 = states[-1], states[-2]
    q, _ = ph.hdm_step(prob, q1, q2, rtol=1e-13)
    d = q - q1
    Phi = (d / np.linalg.norm(d))[:, None]
    hat = np.arange(30, 50)                       # around the waves
    params = pa.HybridParams(eps_y=1e-13, jmax=60)
    out = pa.hybrid_step(prob, q1, q2, Phi, q1, hat, params)
    assert out["l"] == 4 and 2 <= out["J"] <= 60
    assert np.max(np.abs(out["gamma"] - q)) < 1e-10


def test_paper_arom_on_sod():
    """Alg. 1 on Sod's tube (100 cells, 201 steps) with the paper's w = 5,
    m = 4, delta = 0.8 and filters 2, 4, 6 (z = 5): every hybrid snapshot
    stays within 1 % (relative L1) of the full-order state, with fewer
    than half of the cells sampled on hybrid steps and J in [2, j_max]."""
    nx, steps = 100, 201
    prob, q0 = ph.sod(nx, steps)
    hdm = ph.run(prob, q0, steps, rtol=1e-13)
    p = arom.AromParams(w=5, m=4, z=5, rule=sampling.RULE_RRE, delta=0.8, halo=2)
    errs = []
    res = pa.run(prob, q0, steps, p, on_step=lambda k, g, rec: errs.append(arom.relative_l1_error(g, hdm[k])))
    recs = res["records"]
    hyb = [r for r in recs if r["type"] == "hybrid"]
    sbar, sbar_h = arom.sampling_stats(prob, recs)
    assert len(hyb) > 100
    assert max(errs) < 0.01 and np.mean(errs) < 0.005, (max(errs), np.mean(errs))
    assert sbar_h < 0.5 and all(2 <= r["J"] <= 10 for r in hyb)


def test_paper_arom_with_odeim_on_sod():
    """Alg. 1 with the paper's sampled set (hat-S = G u P, n_p = 2 m_eff ODEIM
    points, the fit over them, no halo) on Sod's tube (100 cells, z = 5):
    every hybrid step's sampled set holds the points' cells, and the
    snapshots stay within 1 % of the full-order run."""
    nx, steps = 100, 201
    prob, q0 = ph.sod(nx, steps)
    hdm = ph.run(prob, q0, steps, rtol=1e-13)
    p = arom.AromParams(w=5, m=4, z=5, rule=sampling.RULE_RRE, delta=0.8, halo=0)
    errs = []
    res = pa.run(prob, q0, steps, p, odeim_factor=2,
                 on_step=lambda k, g, rec: errs.append(arom.relative_l1_error(g, hdm[k])))
    hyb = [r for r in res["records"] if r["type"] == "hybrid"]
    assert len(hyb) > 100 and all(r["n_p"] == 8 for r in hyb)
    assert max(errs) < 0.01 and np.mean(errs) < 0.005, (max(errs), np.mean(errs))


def test_paper_filter_moves_a_converged_state_only_below_its_residual():
    """The gated filter sequence on a converged BDF2 state of Sod's tube:
    a filter pass lowers a cell's residual only where the state is already a
    root up to rounding (the implicit solve leaves momenta of 1e-25..1e-54 in
    the constant regions, and the strict gate compares residuals exactly), so
    the state moves by less than its own residual size, nowhere by O(h^2)."""
    prob, states = _sod_states(120, 240, 30)
    q2, q1, q = states[-3], states[-2], states[-1]
    r = pa.cell_residual_norm(prob, q, q1, q2)
    g = pa.spatial_filter(prob, q, q1, q2, pa.HybridParams())
    assert np.max(np.abs(g - q)) <= np.max(r)


def test_paper_filter_removes_a_planted_two_cell_oscillation():
    """A 2-dx oscillation of 1e-3 planted on eight cells of the constant left
    state (all four components) of a converged state: the order-2 pass
    annihilates it in the interior and the gates keep those cells, so the
    filtered state is back at the converged one to 1e-6 of the amplitude and
    the sum of the cell residual norms falls by more than 1e6."""
    prob, states = _sod_states(120, 240, 30)
    q2, q1, q = states[-3], states[-2], states[-1]
    n = prob.ncell
    cells = np.arange(10, 18)
    noisy = q.copy()
    for a in range(4):
        noisy[a * n + cells] += 1e-3 * (1 + a) * (-1.0) ** cells
    log = []
    g = pa.spatial_filter(prob, noisy, q1, q2, pa.HybridParams(), log)
    assert log[0][0] == 1 and log[0][2] >= cells.size
    assert np.max(np.abs(g - q)) < 1e-6 * 4e-3
    r0 = pa.cell_residual_norm(prob, noisy, q1, q2).sum()
    r1 = pa.cell_residual_norm(prob, g, q1, q2).sum()
    assert r1 < 1e-6 * r0
