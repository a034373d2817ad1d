"""Seeded synthetic workloads for the hybrid-snapshot adaptive ROM.

This module only *draws inputs*: grids, initial states and the fixed problem
parameters (cell sizes, time step, ratio of specific heats, boundary type).
It contains none of the method's arithmetic (no flux, residual, solve,
sampling, fit, filter or basis computation), so that both the GPU library's
tests and the CPU oracle can take their inputs from it without sharing any
code of the method.

Workloads (all on the unit square / unit interval, cell centres at
``(i + 1/2) dx``):

* ``burgers1d_1k``   -- 1D inviscid Burgers, 1024 cells, 200 steps, m=10,
  top 10 % sampling, full solve every 20 steps.  u0 = 1 + a sin(2 pi x),
  a ~ U(0.3, 0.6); inflow value u0(0) on the left, outflow on the right.
* ``burgers1d_256k`` -- the same law with 262144 cells, 2000 steps, m=20, 5 %.
* ``burgers2d_1024`` -- 2D scalar Burgers, 1024^2 cells, periodic, 8 Gaussian
  bumps (centres U(0,1)^2, widths U(0.02,0.08), amplitudes U(0.5,1.5)),
  500 steps, m=32, 5 %.
* ``euler2d_512``    -- 2D Euler, gamma=1.4, 512^2 cells, four-quadrant
  Riemann data (rho in [0.1,1.5], p in [0.03,1.5], |u|,|v| <= 1.2),
  transmissive walls, 400 steps, m=40, 8 %.
* ``burgers2d_256``  -- 2D Burgers 256^2, 100 steps (the adjoint workload).

The time step is fixed for the whole run from the initial state: a CFL number
of 0.5 on the largest initial wave speed (for Euler, max(|u|+c, |v|+c) with
c the sound speed of the drawn primitive state).  The window length is
w = ceil(1.5 m), the full-solve period z = 20 and the sampled set is dilated
by 2 cells.  These choices follow the workload statements; the paper's own
experiments use w/m = 5/4 (Sod) and 6/4 (implosion).
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

# Kind codes shared by the C ABI (values fixed in the public header).
BURGERS_1D = 0
BURGERS_2D = 1
EULER_2D = 2

# Boundary codes shared by the C ABI.
BC_INFLOW_OUTFLOW = 0   # left: Dirichlet inflow value; right: zeroth-order extrapolation
BC_PERIODIC = 1
BC_TRANSMISSIVE = 2     # every side: zeroth-order extrapolation (ghost = boundary cell)

KIND_NAMES = {BURGERS_1D: "burgers1d", BURGERS_2D: "burgers2d", EULER_2D: "euler2d"}


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    kind: int
    nx: int
    ny: int
    steps: int
    m: int
    frac: float
    z: int = 20
    halo: int = 2
    checkpoint: int = 0

    @property
    def w(self) -> int:
        return int(math.ceil(1.5 * self.m))

    @property
    def ncomp(self) -> int:
        return 4 if self.kind == EULER_2D else 1

    @property
    def ncell(self) -> int:
        return self.nx * self.ny

    @property
    def n(self) -> int:
        return self.ncomp * self.ncell

    @property
    def bc(self) -> int:
        return {BURGERS_1D: BC_INFLOW_OUTFLOW, BURGERS_2D: BC_PERIODIC,
                EULER_2D: BC_TRANSMISSIVE}[self.kind]

    def resized(self, nx: int, ny: int | None = None, **kw) -> "Workload":
        """Same law, boundary and sampling rule on another grid (for small cases)."""
        if ny is None:
            ny = 1 if self.kind == BURGERS_1D else nx
        return dataclasses.replace(self, nx=nx, ny=ny, **kw)


WORKLOADS = {
    "burgers1d_1k": Workload("burgers1d_1k", BURGERS_1D, 1024, 1, 200, 10, 0.10),
    "burgers1d_256k": Workload("burgers1d_256k", BURGERS_1D, 262144, 1, 2000, 20, 0.05),
    "burgers2d_1024": Workload("burgers2d_1024", BURGERS_2D, 1024, 1024, 500, 32, 0.05),
    "euler2d_512": Workload("euler2d_512", EULER_2D, 512, 512, 400, 40, 0.08),
    "burgers2d_256": Workload("burgers2d_256", BURGERS_2D, 256, 256, 100, 32, 0.05, checkpoint=10),
}

GAMMA = 1.4


@dataclasses.dataclass(frozen=True)
class Problem:
    """Fixed parameters of one run (everything the discretisation needs)."""
    kind: int
    nx: int
    ny: int
    bc: int
    dx: float
    dy: float
    dt: float
    gamma: float
    inflow: float

    @property
    def ncomp(self) -> int:
        return 4 if self.kind == EULER_2D else 1

    @property
    def ncell(self) -> int:
        return self.nx * self.ny

    @property
    def n(self) -> int:
        return self.ncomp * self.ncell


def cell_centres(n: int) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def _burgers1d_u0(wl: Workload, rng: np.random.Generator):
    a = rng.uniform(0.3, 0.6)
    x = cell_centres(wl.nx)
    u0 = 1.0 + a * np.sin(2.0 * np.pi * x)
    inflow = 1.0 + a * math.sin(0.0)
    return u0, inflow


def _burgers2d_u0(wl: Workload, rng: np.random.Generator):
    x = cell_centres(wl.nx)[None, :]
    y = cell_centres(wl.ny)[:, None]
    u0 = np.zeros((wl.ny, wl.nx))
    for _ in range(8):
        cx = rng.uniform(0.0, 1.0)
        cy = rng.uniform(0.0, 1.0)
        width = rng.uniform(0.02, 0.08)
        amp = rng.uniform(0.5, 1.5)
        ddx = np.abs(x - cx)
        ddx = np.minimum(ddx, 1.0 - ddx)          # periodic minimum image
        ddy = np.abs(y - cy)
        ddy = np.minimum(ddy, 1.0 - ddy)
        u0 += amp * np.exp(-(ddx * ddx + ddy * ddy) / (2.0 * width * width))
    return u0.reshape(-1), 0.0


def euler_quadrant_states(rng: np.random.Generator):
    """Primitive (rho, p, u, v) for the NE, NW, SW, SE quadrants, in that order."""
    states = []
    for _ in range(4):
        rho = rng.uniform(0.1, 1.5)
        p = rng.uniform(0.03, 1.5)
        u = rng.uniform(-1.2, 1.2)
        v = rng.uniform(-1.2, 1.2)
        states.append((rho, p, u, v))
    return states


def _euler2d_u0(wl: Workload, rng: np.random.Generator):
    states = euler_quadrant_states(rng)
    x = cell_centres(wl.nx)[None, :] * np.ones((wl.ny, 1))
    y = cell_centres(wl.ny)[:, None] * np.ones((1, wl.nx))
    east = x > 0.5
    north = y > 0.5
    quad = np.where(north & east, 0, np.where(north, 1, np.where(east, 3, 2)))
    prim = np.array(states)                     # (4, 4): rho, p, u, v
    rho = prim[quad, 0]
    p = prim[quad, 1]
    u = prim[quad, 2]
    v = prim[quad, 3]
    energy = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)
    q0 = np.stack([rho, rho * u, rho * v, energy]).reshape(-1)   # component-major
    return q0, 0.0, states


def make(wl: Workload | str, seed: int = 0):
    """Return (problem, q0) for a workload and seed.

    q0 is float64, component-major: q[c * ncell + i + nx * j].
    """
    if isinstance(wl, str):
        wl = WORKLOADS[wl]
    rng = np.random.default_rng(seed)
    dx = 1.0 / wl.nx
    dy = 1.0 / wl.ny if wl.kind != BURGERS_1D else 1.0
    if wl.kind == BURGERS_1D:
        q0, inflow = _burgers1d_u0(wl, rng)
        speed = float(np.max(np.abs(q0)))
    elif wl.kind == BURGERS_2D:
        q0, inflow = _burgers2d_u0(wl, rng)
        speed = float(np.max(np.abs(q0)))
    else:
        q0, inflow, states = _euler2d_u0(wl, rng)
        speed = 0.0
        for rho, p, u, v in states:
            c = math.sqrt(GAMMA * p / rho)
            speed = max(speed, abs(u) + c, abs(v) + c)
    dt = 0.5 * dx / speed
    prob = Problem(kind=wl.kind, nx=wl.nx, ny=wl.ny, bc=wl.bc, dx=dx, dy=dy, dt=dt,
                   gamma=GAMMA, inflow=inflow)
    return prob, np.ascontiguousarray(q0, dtype=np.float64)


# ------------------------------------------------- the paper's experiments
PAPER_BC_FIXED, PAPER_BC_WALL = 0, 1   # HS_PAPER_BC_* (public header)


@dataclasses.dataclass(frozen=True)
class PaperCase:
    """Inputs of an experiment run with the paper's own scheme: mesh, step,
    boundary kind, ghost states (conservative, left/right/bottom/top) and the
    initial state q0 (component-major)."""
    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    dt: float
    steps: int
    gamma: float
    bc: int
    ghost: tuple
    q0: np.ndarray


def _conservative(rho, u, v, p):
    return np.stack([rho, rho * u, rho * v, p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)])


def paper_sod(nx: int = 499, steps: int = 999, T: float = 0.2) -> PaperCase:
    """Sod's shock tube (Sec. 3.2): (0, 1), (rho, u, P) = (1, 0, 1) left of
    0.5 and (0.125, 0, 0.1) right of it, T = 0.2, N = 499 cells and
    N_t = 999 steps by default; ghosts hold the initial boundary states."""
    x = cell_centres(nx)
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    q = _conservative(rho, 0 * x, 0 * x, p)
    ghost = (tuple(q[:, 0]), tuple(q[:, -1]), tuple(q[:, 0]), tuple(q[:, 0]))
    return PaperCase("sod", nx, 1, 1.0 / nx, 1.0, T / steps, steps, GAMMA, PAPER_BC_FIXED, ghost,
                     np.ascontiguousarray(q.reshape(-1)))


def paper_implosion(n: int = 100, steps: int = 1650, T: float = 0.5) -> PaperCase:
    """The model implosion (Sec. 3.3): (0, 0.3)^2 with reflective walls,
    (rho, P) = (0.125, 0.14) where x_1 + x_2 <= 0.15 and (1, 1) elsewhere, at
    rest; T = 0.5 over 1650 steps on 100^2 cells by default."""
    h = 0.3 / n
    c = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(c, c)                      # row j = y, column i = x
    inner = (X + Y <= 0.15).reshape(-1)
    rho = np.where(inner, 0.125, 1.0)
    p = np.where(inner, 0.14, 1.0)
    z = np.zeros(n * n)
    q = _conservative(rho, z, z, p)
    return PaperCase("implosion", n, n, h, h, T / steps, steps, GAMMA, PAPER_BC_WALL, (),
                     np.ascontiguousarray(q.reshape(-1)))


def random_euler_state(nx: int, ny: int, seed: int, mach: float = 0.8) -> np.ndarray:
    """Seeded cell-wise random Euler states: rho in [0.5, 1.5], P in
    [0.3, 1.3], velocity components up to mach times the sound speed."""
    rng = np.random.default_rng(seed)
    n = nx * ny
    rho = 0.5 + rng.random(n)
    p = 0.3 + rng.random(n)
    c = np.sqrt(GAMMA * p / rho)
    u = mach * c * (2 * rng.random(n) - 1)
    v = mach * c * (2 * rng.random(n) - 1) if ny > 1 else 0 * u
    return np.ascontiguousarray(_conservative(rho, u, v, p).reshape(-1))


def random_unit_vectors(n: int, count: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) directions, normalised (for finite-difference checks)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((count, n))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
