"""The paper's own high-dimensional model (oracle; test use only).

Sec. 3.1 discretises the Euler equations (eq. euler, ideal gas) by a finite
volume method on a Cartesian mesh: second-order MUSCL reconstruction with the
minmod limiter and Roe's approximate Riemann solver for the face fluxes, and
BDF2 in time (eq. bdf with a_0 = 1/3, a_1 = -4/3, a_2 = 1, beta = 2/3), the
residual of eq. hdm:

    R_k(q) = q - (2/3) dt f*(q) + (1/3) q_{k-2} - (4/3) q_{k-1} .

Readings where the paper is silent (listed in the design notes):
* MUSCL reconstructs the primitive variables (rho, u, v, P) cell by cell,
  slope minmod(w_i - w_{i-1}, w_{i+1} - w_i); the face states are
  w_i + slope_i / 2 and w_{i+1} - slope_{i+1} / 2.
* Roe's solver without an entropy fix (Sod's rarefaction is not transonic).
* Boundaries: "suitable boundary conditions from the initial condition"
  (Sec. 3.2): two ghost cells on each side hold the initial state of the
  boundary cell (held fixed); or reflective walls (mirror state, normal
  velocity negated) where a problem asks for them.
* The first step has no q_{k-2}: it is BDF1 (q - dt f*(q) - q_{k-1}).
* Newton on a finite-difference Jacobian (columns grouped by colour, the
  stencil reaches two cells along each axis): the limiter's kinks rule out
  complex steps; the iteration stops at ||R||_inf <= 1e-12 max(1, |q|_inf).

State layout as in oracle.fv: q = (rho, rho u, rho v, E), component-major
over cells i + nx j.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

BDF2 = (1.0 / 3.0, -4.0 / 3.0, 1.0, 2.0 / 3.0)    # a_0, a_1, a_2, beta (eq. bdf, Sec. 3.1)
FIXED, WALL = 0, 1                                 # ghosts from given states; reflective walls


@dataclass(frozen=True)
class PaperProblem:
    nx: int
    ny: int
    dx: float
    dy: float
    dt: float
    gamma: float
    bc: int = FIXED                      # FIXED: ghosts from the initial state; WALL: reflective
    ghost: tuple = ()                    # FIXED: (left, right[, bottom, top]) conservative 4-vectors

    @property
    def ncell(self):
        return self.nx * self.ny

    @property
    def n(self):
        return 4 * self.ncell


def minmod(a, b):
    """0 where a and b differ in sign (or one is 0), else the one of smaller
    magnitude."""
    return np.where(a * b > 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def primitive(q, gamma):
    rho, mx, my, en = q
    u, v = mx / rho, my / rho
    p = (gamma - 1.0) * (en - 0.5 * rho * (u * u + v * v))
    return np.stack([rho, u, v, p])


def conservative(w, gamma):
    rho, u, v, p = w
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def physical_flux(q, gamma, axis):
    """Euler flux along axis 0 (x) or 1 (y) of conservative states q (4, ...)."""
    rho, u, v, p = primitive(q, gamma)
    en = q[3]
    if axis == 0:
        return np.stack([rho * u, rho * u * u + p, rho * u * v, (en + p) * u])
    return np.stack([rho * v, rho * u * v, rho * v * v + p, (en + p) * v])


def roe_waves(qL, qR, gamma, axis):
    """Roe's linearisation between qL and qR along an axis: wave speeds
    lambda_k, strengths alpha_k and right eigenvectors r_k (k = 1..4: the
    acoustic wave u_n - c, the entropy wave, the shear wave, u_n + c), with
    the Roe-averaged velocity, enthalpy and sound speed."""
    rL, uL, vL, pL = primitive(qL, gamma)
    rR, uR, vR, pR = primitive(qR, gamma)
    HL = (qL[3] + pL) / rL
    HR = (qR[3] + pR) / rR
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    rt = sL * sR
    ut = (sL * uL + sR * uR) / (sL + sR)
    vt = (sL * vL + sR * vR) / (sL + sR)
    Ht = (sL * HL + sR * HR) / (sL + sR)
    ct = np.sqrt((gamma - 1.0) * (Ht - 0.5 * (ut * ut + vt * vt)))
    un, us = (ut, vt) if axis == 0 else (vt, ut)
    dr, dp = rR - rL, pR - pL
    dun, dus = ((uR - uL), (vR - vL)) if axis == 0 else ((vR - vL), (uR - uL))
    alpha = [(dp - rt * ct * dun) / (2.0 * ct * ct), dr - dp / (ct * ct), rt * dus,
             (dp + rt * ct * dun) / (2.0 * ct * ct)]
    lam = [un - ct, un, un, un + ct]
    one, zero = np.ones_like(ut), np.zeros_like(ut)
    kin = 0.5 * (ut * ut + vt * vt)
    if axis == 0:
        r = [np.stack([one, ut - ct, vt, Ht - ut * ct]), np.stack([one, ut, vt, kin]),
             np.stack([zero, zero, one, vt]), np.stack([one, ut + ct, vt, Ht + ut * ct])]
    else:
        r = [np.stack([one, ut, vt - ct, Ht - vt * ct]), np.stack([one, ut, vt, kin]),
             np.stack([zero, one, zero, ut]), np.stack([one, ut, vt + ct, Ht + vt * ct])]
    return lam, alpha, r


def roe_flux(qL, qR, gamma, axis):
    """F = (F(qL) + F(qR)) / 2 - (1/2) sum_k |lambda_k| alpha_k r_k."""
    lam, alpha, r = roe_waves(qL, qR, gamma, axis)
    f = 0.5 * (physical_flux(qL, gamma, axis) + physical_flux(qR, gamma, axis))
    for k in range(4):
        f = f - 0.5 * np.abs(lam[k]) * alpha[k] * r[k]
    return f


def _padded(prob: PaperProblem, q):
    """The state (4, ny + 4, nx + 4) with two ghost layers on every side."""
    g = q.reshape(4, prob.ny, prob.nx)
    if prob.bc == WALL:
        gx = np.pad(g, ((0, 0), (0, 0), (2, 2)), mode="symmetric")
        gx[1, :, :2] *= -1.0                     # the wall's normal velocity changes sign
        gx[1, :, -2:] *= -1.0
        if prob.ny == 1:
            return np.pad(gx, ((0, 0), (2, 2), (0, 0)), mode="edge")
        gy = np.pad(gx, ((0, 0), (2, 2), (0, 0)), mode="symmetric")
        gy[2, :2, :] *= -1.0
        gy[2, -2:, :] *= -1.0
        return gy
    left, right = prob.ghost[0], prob.ghost[1]
    out = np.empty((4, prob.ny + 4, prob.nx + 4))
    out[:, 2:-2, 2:-2] = g
    out[:, 2:-2, :2] = np.asarray(left)[:, None, None]
    out[:, 2:-2, -2:] = np.asarray(right)[:, None, None]
    if prob.ny == 1:
        out[:, :2, :] = out[:, 2:3, :]
        out[:, -2:, :] = out[:, -3:-2, :]
    else:
        bottom, top = prob.ghost[2], prob.ghost[3]
        out[:, :2, :] = np.asarray(bottom)[:, None, None]
        out[:, -2:, :] = np.asarray(top)[:, None, None]
    return out


def face_fluxes(prob: PaperProblem, q, axis):
    """Roe fluxes on the faces along an axis, from MUSCL-minmod states of the
    primitive variables: (4, ny, nx + 1) for x, (4, ny + 1, nx) for y."""
    P = _padded(prob, q)
    w = primitive(P, prob.gamma)
    if axis == 0:
        w = w[:, 2:-2, :]                                   # (4, ny, nx + 4)
        slope = minmod(w[:, :, 1:-1] - w[:, :, :-2], w[:, :, 2:] - w[:, :, 1:-1])   # cells -1 .. nx
        wc = w[:, :, 1:-1]
        wL = wc[:, :, :-1] + 0.5 * slope[:, :, :-1]         # faces -1/2 .. nx - 1/2
        wR = wc[:, :, 1:] - 0.5 * slope[:, :, 1:]
    else:
        w = w[:, :, 2:-2]                                   # (4, ny + 4, nx)
        slope = minmod(w[:, 1:-1, :] - w[:, :-2, :], w[:, 2:, :] - w[:, 1:-1, :])
        wc = w[:, 1:-1, :]
        wL = wc[:, :-1, :] + 0.5 * slope[:, :-1, :]
        wR = wc[:, 1:, :] - 0.5 * slope[:, 1:, :]
    return roe_flux(conservative(wL, prob.gamma), conservative(wR, prob.gamma), prob.gamma, axis)


def rhs(prob: PaperProblem, q):
    """f*(q): minus the flux divergence of every cell (eq. semi_disc)."""
    fx = face_fluxes(prob, q, 0)
    out = -(fx[:, :, 1:] - fx[:, :, :-1]) / prob.dx
    if prob.ny > 1:
        fy = face_fluxes(prob, q, 1)
        out = out - (fy[:, 1:, :] - fy[:, :-1, :]) / prob.dy
    return out.reshape(-1)


def residual(prob: PaperProblem, q, q1, q2=None):
    """eq. hdm with BDF2 (q1 = q_{k-1}, q2 = q_{k-2}); BDF1 when q2 is None."""
    if q2 is None:
        return q - prob.dt * rhs(prob, q) - q1
    a0, a1, a2, beta = BDF2
    return a2 * q - prob.dt * beta * rhs(prob, q) + a0 * q2 + a1 * q1


def fd_jacobian(prob: PaperProblem, q, q1, q2=None):
    """dR/dq by forward differences; the columns of cells five apart along
    each axis (and each component separately) share one residual evaluation."""
    n = prob.n
    R0 = residual(prob, q, q1, q2)
    rows, cols, vals = [], [], []
    cx = np.arange(prob.nx)[None, :] % 5
    cy = np.arange(prob.ny)[:, None] % 5 if prob.ny > 1 else np.zeros((1, 1), int)
    colour = (cx + 5 * cy).reshape(-1)
    for a in range(4):
        for c in np.unique(colour):
            cells = np.flatnonzero(colour == c)
            idx = a * prob.ncell + cells
            h = 1e-7 * np.maximum(1.0, np.abs(q[idx]))
            qp = q.copy()
            qp[idx] += h
            dR = residual(prob, qp, q1, q2) - R0
            # each perturbed cell owns the rows of the cells within two of it
            gi, gj = cells % prob.nx, cells // prob.nx
            for di in range(-2, 3):
                for dj in (range(-2, 3) if prob.ny > 1 else (0,)):
                    ri, rj = gi + di, gj + dj
                    ok = (ri >= 0) & (ri < prob.nx) & (rj >= 0) & (rj < prob.ny)
                    rc = ri[ok] + prob.nx * rj[ok]
                    for b in range(4):
                        rows.append(b * prob.ncell + rc)
                        cols.append(idx[ok])
                        vals.append(dR[b * prob.ncell + rc] / h[ok])
    return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def hdm_step(prob: PaperProblem, q1, q2=None, maxit=30, rtol=1e-12):
    """One time step: Newton on eq. hdm from q_{k-1} until
    ||R||_inf <= rtol max(1, |q_{k-1}|_inf); returns (q_k, iterations)."""
    q = q1.copy()
    tol = rtol * max(1.0, float(np.max(np.abs(q1))))
    for it in range(maxit + 1):
        R = residual(prob, q, q1, q2)
        if np.max(np.abs(R)) <= tol:
            return q, it
        if it == maxit:
            break
        q = q - spla.spsolve(fd_jacobian(prob, q, q1, q2), R)
    raise RuntimeError("Newton on the paper's HDM did not converge")


def run(prob: PaperProblem, q0, steps, rtol=1e-12):
    """N_t steps: BDF1 for the first, BDF2 after; returns every state."""
    states = [q0.copy()]
    for k in range(steps):
        q2 = states[-2] if k >= 1 else None
        q, _ = hdm_step(prob, states[-1], q2, rtol=rtol)
        states.append(q)
    return states


def sod(nx, steps, T=0.2, gamma=1.4):
    """Sod's shock tube (Sec. 3.2): (0, 1), interface at 0.5, left (1, 0, 1),
    right (0.125, 0, 0.1), ghosts from the initial state; returns (prob, q0)."""
    x = (np.arange(nx) + 0.5) / nx
    left = x < 0.5
    w = np.stack([np.where(left, 1.0, 0.125), 0.0 * x, 0.0 * x, np.where(left, 1.0, 0.1)])
    q0 = conservative(w, gamma).reshape(-1)
    ghost = (conservative(w[:, :1], gamma)[:, 0], conservative(w[:, -1:], gamma)[:, 0])
    prob = PaperProblem(nx=nx, ny=1, dx=1.0 / nx, dy=1.0, dt=T / steps, gamma=gamma, bc=FIXED, ghost=ghost)
    return prob, q0
