"""Pins of the oracle's finite-volume HDM against facts the paper and the
mathematics fix (no GPU): conservation with boundary fluxes, the
Rankine-Hugoniot shock speed, fixed points, the characteristic solution of
smooth Burgers data, the exact Riemann solution of Sod's shock tube (the
paper's first experiment), reduction of y-uniform Euler data to one
dimension, x/y transpose symmetry, finite-difference Jacobians and Newton's
quadratic convergence."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import fv

HERE = os.path.dirname(__file__)


def burgers1d(nx, u0, inflow, cfl_speed=None, bc=W.BC_INFLOW_OUTFLOW):
    speed = cfl_speed or float(np.max(np.abs(u0)))
    dx = 1.0 / nx
    return W.Problem(kind=W.BURGERS_1D, nx=nx, ny=1, bc=bc, dx=dx, dy=1.0,
                     dt=0.5 * dx / speed, gamma=1.4, inflow=inflow)


def euler(nx, ny, dt, bc=W.BC_TRANSMISSIVE):
    return W.Problem(kind=W.EULER_2D, nx=nx, ny=ny, bc=bc, dx=1.0 / nx, dy=1.0 / ny,
                     dt=dt, gamma=1.4, inflow=0.0)


def prim_to_cons(rho, u, v, p, g=1.4):
    return np.concatenate([rho, rho * u, rho * v, p / (g - 1) + 0.5 * rho * (u * u + v * v)])


def euler_physical_flux_x(q, g=1.4):
    rho, mx, my, E = q
    u, v = mx / rho, my / rho
    p = (g - 1) * (E - 0.5 * rho * (u * u + v * v))
    return np.array([rho * u, rho * u * u + p, rho * u * v, u * (E + p)])


# ---------------------------------------------------------------- conservation

def test_conservation_periodic_burgers2d():
    wl = W.WORKLOADS["burgers2d_1024"].resized(40, 36)
    prob, q = W.make(wl, 3)
    for _ in range(5):
        qn, _ = fv.hdm_step(prob, q)
        tol = fv.newton_tol(q)
        assert abs(np.sum(qn) - np.sum(q)) <= prob.n * tol
        q = qn


def test_conservation_inflow_outflow_burgers1d():
    wl = W.WORKLOADS["burgers1d_1k"].resized(300)
    prob, q = W.make(wl, 1)
    lx = prob.dt / prob.dx
    for _ in range(5):
        qn, _ = fv.hdm_step(prob, q)
        # boundary fluxes of the new state: inflow face (ghost = inflow value)
        # and the outflow face, where both states equal the last cell: f(u) = u^2/2
        uL, u0 = prob.inflow, qn[0]
        f_in = 0.25 * (uL ** 2 + u0 ** 2) - 0.5 * max(abs(uL), abs(u0)) * (u0 - uL)
        f_out = 0.5 * qn[-1] ** 2
        balance = np.sum(qn - q) + lx * (f_out - f_in)
        assert abs(balance) <= prob.n * fv.newton_tol(q)
        q = qn


def test_conservation_periodic_euler():
    nx, ny = 24, 20
    rng = np.random.default_rng(5)
    X, Y = np.meshgrid((np.arange(nx) + .5) / nx, (np.arange(ny) + .5) / ny)
    rho = (1 + 0.3 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)).ravel()
    u = (0.3 * np.cos(2 * np.pi * Y)).ravel()
    v = (0.2 * np.sin(2 * np.pi * X)).ravel()
    p = (1 + 0.2 * rng.random(nx * ny)).ravel()
    q = prim_to_cons(rho, u, v, p)
    prob = euler(nx, ny, 0.4 / nx / 1.6, W.BC_PERIODIC)
    for _ in range(3):
        qn, _ = fv.hdm_step(prob, q)
        for c in range(4):
            s = slice(c * nx * ny, (c + 1) * nx * ny)
            assert abs(np.sum(qn[s]) - np.sum(q[s])) <= prob.ncell * fv.newton_tol(q)
        q = qn


def test_conservation_transmissive_euler_with_boundary_fluxes():
    prob, q = W.make(W.WORKLOADS["euler2d_512"].resized(20, 16), 2)
    nx, ny, nc = prob.nx, prob.ny, prob.ncell
    qn, _ = fv.hdm_step(prob, q)
    g = qn.reshape(4, ny, nx)
    # physical fluxes at the four walls (ghost = boundary cell, so F(q,q) = f(q))
    fx = lambda col: euler_physical_flux_x(g[:, :, col])
    swap = [0, 2, 1, 3]
    fy = lambda row: euler_physical_flux_x(g[swap][:, row, :])[swap]
    out_x = (fx(nx - 1) - fx(0)).sum(axis=1) * prob.dt / prob.dx
    out_y = (fy(ny - 1) - fy(0)).sum(axis=1) * prob.dt / prob.dy
    for c in range(4):
        s = slice(c * nc, (c + 1) * nc)
        bal = np.sum(qn[s] - q[s]) + out_x[c] + out_y[c]
        assert abs(bal) <= 4 * nc * fv.newton_tol(q), (c, bal)


# ---------------------------------------------------------------- Rankine-Hugoniot

@pytest.mark.parametrize("uL,uR", [(1.5, 0.5), (1.2, -0.4)])
def test_rankine_hugoniot_mass_equivalent_shock(uL, uR):
    nx = 400
    x = (np.arange(nx) + 0.5) / nx
    x0 = 0.3
    q = np.where(x < x0, uL, uR).astype(float)
    prob = burgers1d(nx, q, inflow=uL)
    s = 0.5 * (uL + uR)
    t = 0.0
    for _ in range(60):
        q, _ = fv.hdm_step(prob, q)
        t += prob.dt
    mass = np.sum(q) * prob.dx
    xs = (mass - uR * 1.0) / (uL - uR)
    assert abs(xs - (x0 + s * t)) < 1e-11


# ---------------------------------------------------------------- fixed points

@pytest.mark.parametrize("name", ["burgers1d_1k", "burgers2d_1024", "euler2d_512"])
def test_constant_state_is_fixed_point(name):
    wl = W.WORKLOADS[name].resized(12)
    prob, q0 = W.make(wl, 0)
    const = np.concatenate([np.full(prob.ncell, q0[c * prob.ncell]) for c in range(prob.ncomp)])
    if prob.bc == W.BC_INFLOW_OUTFLOW:
        prob = W.Problem(**{**prob.__dict__, "inflow": const[0]})
    R = fv.residual(prob, const, const)
    assert np.all(R == 0.0)
    q, its = fv.hdm_step(prob, const)
    assert its == 0 and np.array_equal(q, const)


# ---------------------------------------------------------------- smooth Burgers

def characteristic_solution(x, t, a):
    """u = u0(x - u t) with u0 = 1 + a sin(2 pi x) for x >= 0 and the inflow
    value 1 for x < 0 (before breaking, t < 1/(2 pi a))."""
    u0 = lambda s: np.where(s >= 0, 1.0 + a * np.sin(2 * np.pi * s), 1.0)
    du0 = lambda s: np.where(s >= 0, 2 * np.pi * a * np.cos(2 * np.pi * s), 0.0)
    u = u0(x)
    for _ in range(60):
        g = u - u0(x - u * t)
        u = u - g / (1.0 + du0(x - u * t) * t)
    return u


def test_burgers_converges_to_characteristic_solution_first_order():
    a, T = 0.45, 0.1
    errs = []
    for nx in (128, 256, 512, 1024):
        x = (np.arange(nx) + 0.5) / nx
        q = 1.0 + a * np.sin(2 * np.pi * x)
        dx = 1.0 / nx
        steps = int(math.ceil(T / (0.5 * dx / (1 + a))))
        prob = W.Problem(kind=W.BURGERS_1D, nx=nx, ny=1, bc=W.BC_INFLOW_OUTFLOW, dx=dx,
                         dy=1.0, dt=T / steps, gamma=1.4, inflow=1.0)
        for _ in range(steps):
            q, _ = fv.hdm_step(prob, q)
        errs.append(np.sum(np.abs(q - characteristic_solution(x, T, a))) * dx)
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(0.85 < o < 1.15 for o in orders), (errs, orders)


# ---------------------------------------------------------------- Sod (paper Sec. 3.2)

def exact_riemann(left, right, g, xi):
    """Exact Riemann solution of the 1D Euler equations for an ideal gas
    (two-rarefaction / two-shock pressure function, Newton on p*), sampled at
    xi = (x - x0)/t.  Returns (rho, u, p, p_star, u_star)."""
    rL, uL, pL = left
    rR, uR, pR = right
    cL, cR = math.sqrt(g * pL / rL), math.sqrt(g * pR / rR)

    def fk(p, rk, pk, ck):
        if p > pk:
            A, B = 2 / ((g + 1) * rk), (g - 1) / (g + 1) * pk
            return (p - pk) * math.sqrt(A / (p + B)), math.sqrt(A / (B + p)) * (1 - (p - pk) / (2 * (B + p)))
        return (2 * ck / (g - 1) * ((p / pk) ** ((g - 1) / (2 * g)) - 1),
                (p / pk) ** (-(g + 1) / (2 * g)) / (rk * ck))

    p = 0.5 * (pL + pR)
    for _ in range(100):
        fL, dL = fk(p, rL, pL, cL)
        fR, dR = fk(p, rR, pR, cR)
        p = max(p - (fL + fR + uR - uL) / (dL + dR), 1e-12)
    ps = p
    us = 0.5 * (uL + uR) + 0.5 * (fk(ps, rR, pR, cR)[0] - fk(ps, rL, pL, cL)[0])
    gm = (g - 1) / (g + 1)
    out = np.empty((3, xi.size))
    for i, s in enumerate(xi):
        if s <= us:
            if ps > pL:
                SL = uL - cL * math.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
                st = (rL, uL, pL) if s < SL else (rL * (ps / pL + gm) / (gm * ps / pL + 1), us, ps)
            else:
                SH, ST = uL - cL, us - cL * (ps / pL) ** ((g - 1) / (2 * g))
                if s < SH:
                    st = (rL, uL, pL)
                elif s > ST:
                    st = (rL * (ps / pL) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) * (cL + (g - 1) / 2 * (uL - s))
                    st = (rL * (c / cL) ** (2 / (g - 1)), 2 / (g + 1) * (cL + (g - 1) / 2 * uL + s),
                          pL * (c / cL) ** (2 * g / (g - 1)))
        else:
            if ps > pR:
                SR = uR + cR * math.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
                st = (rR, uR, pR) if s > SR else (rR * (ps / pR + gm) / (gm * ps / pR + 1), us, ps)
            else:
                SH, ST = uR + cR, us + cR * (ps / pR) ** ((g - 1) / (2 * g))
                if s > SH:
                    st = (rR, uR, pR)
                elif s < ST:
                    st = (rR * (ps / pR) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) * (cR - (g - 1) / 2 * (uR - s))
                    st = (rR * (c / cR) ** (2 / (g - 1)), 2 / (g + 1) * (-cR + (g - 1) / 2 * uR + s),
                          pR * (c / cR) ** (2 * g / (g - 1)))
        out[:, i] = st
    return out[0], out[1], out[2], ps, us


def test_exact_riemann_solver_reproduces_textbook_sod_star_state():
    sod = json.load(open(os.path.join(HERE, "golden", "paper_parameters.json")))["sod"]
    *_, ps, us = exact_riemann(sod["left"], sod["right"], 1.4, np.array([0.0]))
    # star state of Sod's problem to the 5 digits commonly tabulated
    assert abs(ps - 0.30313) < 5e-6 and abs(us - 0.92745) < 5e-6


def test_euler_sod_converges_to_exact_riemann_solution():
    sod = json.load(open(os.path.join(HERE, "golden", "paper_parameters.json")))["sod"]
    errs = []
    for nx in (100, 400):
        x = (np.arange(nx) + 0.5) / nx
        left = x < sod["x0"]
        rho = np.where(left, sod["left"][0], sod["right"][0])
        p = np.where(left, sod["left"][2], sod["right"][2])
        q = prim_to_cons(rho, 0 * x, 0 * x, p)
        cmax = math.sqrt(1.4 * 1.0 / 1.0)
        steps = int(math.ceil(sod["T"] / (0.5 / nx / cmax)))
        prob = euler(nx, 1, sod["T"] / steps)
        for _ in range(steps):
            q, _ = fv.hdm_step(prob, q)
        re, ue, pe, *_ = exact_riemann(sod["left"], sod["right"], 1.4, (x - sod["x0"]) / sod["T"])
        errs.append(np.mean(np.abs(q[:nx] - re)))
    assert errs[1] < 0.025 and errs[0] / errs[1] > 1.6, errs


# ---------------------------------------------------------------- Euler reductions

def test_euler_y_uniform_reduces_to_one_dimension():
    prob2, q2 = W.make(W.WORKLOADS["euler2d_512"].resized(32, 8), 4)
    g = q2.reshape(4, 8, 32).copy()
    g[:, :, :] = g[:, :1, :]           # y-uniform
    g[2] = 0.0                          # v = 0
    q2 = g.reshape(-1)
    prob1 = W.Problem(**{**prob2.__dict__, "ny": 1, "dy": 1.0})
    q1 = g[:, 0, :].reshape(-1)
    for _ in range(3):
        q2, _ = fv.hdm_step(prob2, q2)
        q1, _ = fv.hdm_step(prob1, q1)
    g2 = q2.reshape(4, 8, 32)
    # the sparse LU mixes components, so these hold to rounding, not bitwise
    assert np.max(np.abs(g2[2])) < 1e-15
    assert np.max(np.abs(g2 - g2[:, :1, :])) < 1e-13
    assert np.max(np.abs(g2[:, 0, :].reshape(-1) - q1)) < 1e-12


def test_euler_transpose_symmetry():
    prob, q = W.make(W.WORKLOADS["euler2d_512"].resized(16, 16), 6)
    g = q.reshape(4, 16, 16)
    gt = g.transpose(0, 2, 1)[[0, 2, 1, 3]].copy()
    a, _ = fv.hdm_step(prob, q)
    b, _ = fv.hdm_step(prob, gt.reshape(-1))
    at = a.reshape(4, 16, 16).transpose(0, 2, 1)[[0, 2, 1, 3]]
    assert np.max(np.abs(at.reshape(-1) - b)) < 1e-13


def test_euler_positivity_on_workload():
    prob, q = W.make(W.WORKLOADS["euler2d_512"].resized(24), 1)
    for _ in range(4):
        q, _ = fv.hdm_step(prob, q)
        g = q.reshape(4, -1)
        p = 0.4 * (g[3] - 0.5 * (g[1] ** 2 + g[2] ** 2) / g[0])
        assert np.all(g[0] > 0) and np.all(p > 0)


# ---------------------------------------------------------------- Jacobian / Newton

CASES = [("burgers1d_1k", 9, 1), ("burgers2d_1024", 7, 2), ("euler2d_512", 5, 3)]


@pytest.mark.parametrize("name,nx,seed", CASES)
def test_jacobian_matches_central_differences(name, nx, seed):
    wl = W.WORKLOADS[name].resized(nx)
    prob, q0 = W.make(wl, seed)
    rng = np.random.default_rng(seed)
    q = q0 * (1 + 0.05 * rng.standard_normal(q0.size))
    if prob.kind == W.BURGERS_2D:
        # keep states off u = 0 and neighbours well apart: |u| and the max() in the
        # wave speed have kinks that a finite-difference step must not straddle
        q = q + 0.3 + 0.2 * rng.random(q.size)
    J = fv.jacobian(prob, q).toarray()
    h = 1e-6
    Jfd = np.empty_like(J)
    for j in range(q.size):
        e = np.zeros(q.size)
        e[j] = h * max(1.0, abs(q[j]))
        Jfd[:, j] = (fv.residual(prob, q + e, q0) - fv.residual(prob, q - e, q0)) / (2 * e[j])
    assert np.max(np.abs(J - Jfd)) < 1e-7 * max(1.0, np.max(np.abs(J)))


def test_jacobian_periodic_euler_matches_central_differences():
    prob = euler(5, 4, 0.05, W.BC_PERIODIC)
    _, q0 = W.make(W.WORKLOADS["euler2d_512"].resized(5, 4), 7)
    # break the equal face states of the piecewise-constant data (a tie in the
    # wave-speed max is a kink the finite-difference step would straddle)
    q0 = q0 * (1 + 0.05 * np.random.default_rng(7).standard_normal(q0.size))
    J = fv.jacobian(prob, q0).toarray()
    h = 1e-6
    for j in range(q0.size):
        e = np.zeros(q0.size)
        e[j] = h * max(1.0, abs(q0[j]))
        col = (fv.residual(prob, q0 + e, q0) - fv.residual(prob, q0 - e, q0)) / (2 * e[j])
        assert np.max(np.abs(J[:, j] - col)) < 1e-7 * max(1.0, np.max(np.abs(J)))


@pytest.mark.parametrize("name,nx,seed", CASES)
def test_newton_converges_quadratically(name, nx, seed):
    wl = W.WORKLOADS[name].resized(max(nx, 16))
    prob, q0 = W.make(wl, seed)
    prob = W.Problem(**{**prob.__dict__, "dt": prob.dt * 8})   # harder step
    q = q0.copy()
    norms = []
    import scipy.sparse.linalg as spla
    for _ in range(12):
        R = fv.residual(prob, q, q0)
        norms.append(np.max(np.abs(R)))
        if norms[-1] < 1e-13:
            break
        q = q - spla.spsolve(fv.jacobian(prob, q).tocsc(), R)
    k = [i for i in range(1, len(norms)) if norms[i] > 1e-11 and norms[i - 1] < 1e-2]
    for i in k:
        assert norms[i] < 50 * norms[i - 1] ** 2, norms
    assert norms[-1] < 1e-13


@pytest.mark.parametrize("name,nx,ny", [("burgers1d_1k", 300, 1), ("burgers2d_1024", 40, 36), ("euler2d_512", 24, 20)])
def test_jacobian_restricted_rows_equal_full_rows(name, nx, ny):
    """The restricted assembly used by the partial Newton solve gives the
    full Jacobian's entries on the chosen rows, bit for bit."""
    prob, q0 = W.make(W.WORKLOADS[name].resized(nx, ny), 0)
    q1 = fv.hdm_step(prob, q0)[0]
    cells = np.sort(np.random.default_rng(1).choice(prob.ncell, prob.ncell // 5, replace=False))
    d = fv.dofs_of_cells(prob, cells)
    A = fv.jacobian(prob, q1)[d]
    B = fv.jacobian(prob, q1, cells=cells)[d]
    assert np.array_equal(A.toarray(), B.toarray())
