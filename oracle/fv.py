"""Finite-volume HDM: residual, Jacobian and Newton solve (oracle; test use only).

Paper passages followed
-----------------------
* Conservation law and its semi-discretisation: Sec. 2.1 (eq. cons) and
  Sec. 2.2 (eq. semi_disc).
* BDF time discretisation, first order here (backward Euler: a_0 = -1,
  a_1 = 1, beta = 1), eq. bdf; the fully discrete residual
  R_k(q) = q - F_k(q), eq. hdm.
* Euler equations with the ideal-gas law: Sec. 3.1, eq. euler.
* Newton's method for the HDM solve: Sec. 2.4.3 (computational efficiency).

Readings (the paper uses MUSCL + Roe + minmod with BDF2; the workloads here
specify a Rusanov flux with backward Euler):
* piecewise-constant face states (first order, stencil radius 1);
* Rusanov flux F = (f(qL) + f(qR))/2 - alpha/2 (qR - qL), alpha the larger
  spectral radius of the two sides (Burgers |u|; Euler |u_n| + c); a tie
  |aL| = |aR| takes the left branch, |x| at x = 0 takes the + branch;
* ghost cells: periodic wrap; inflow Dirichlet value (left, 1D Burgers);
  zeroth-order extrapolation (outflow / transmissive);
* Newton stops when ||R||_inf <= 1e-13 max(1, ||q_prev||_inf), at most 30
  iterations; each linear system is solved by a sparse direct solve.

Every function accepts complex arrays so that the face-flux derivatives can be
taken by the complex-step method (exact to rounding); branches (abs, max)
are decided on real parts.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import (BURGERS_1D, BURGERS_2D, EULER_2D, BC_INFLOW_OUTFLOW,
                       BC_PERIODIC, BC_TRANSMISSIVE, Problem)

NEWTON_RTOL = 1e-13
NEWTON_MAXIT = 30


class NotConverged(RuntimeError):
    pass


def cabs(x):
    """|x| with the branch decided on the real part (+ branch at 0)."""
    return np.where(np.real(x) >= 0, x, -x)


def cmax(a, b):
    """max(a, b) decided on real parts; a tie returns the first argument."""
    return np.where(np.real(a) >= np.real(b), a, b)


# --------------------------------------------------------------------------
# Face fluxes
# --------------------------------------------------------------------------

def burgers_flux(uL, uR):
    """Rusanov flux of f(u) = u^2/2 between left and right states."""
    a = cmax(cabs(uL), cabs(uR))
    return 0.25 * (uL * uL + uR * uR) - (0.5 * a) * (uR - uL)


def euler_phys(q, gamma, normal):
    """Physical Euler flux along axis ``normal`` (1 = x, 2 = y), the normal
    velocity and the sound speed, for conservative q = (rho, rho u, rho v, E)."""
    rho, mx, my, en = q[0], q[1], q[2], q[3]
    u = mx / rho
    v = my / rho
    p = (gamma - 1.0) * (en - 0.5 * (mx * u + my * v))
    c = np.sqrt(gamma * p / rho)
    if normal == 1:
        un = u
        f = [mx, mx * u + p, my * u, (en + p) * u]
    else:
        un = v
        f = [my, mx * v, my * v + p, (en + p) * v]
    return f, un, c


def euler_flux(qL, qR, gamma, normal):
    fL, unL, cL = euler_phys(qL, gamma, normal)
    fR, unR, cR = euler_phys(qR, gamma, normal)
    a = cmax(cabs(unL) + cL, cabs(unR) + cR)
    out = []
    for k in range(4):
        out.append(0.5 * (fL[k] + fR[k]) - (0.5 * a) * (qR[k] - qL[k]))
    return np.stack(out)


# --------------------------------------------------------------------------
# Grid helpers: states on both sides of every face, ghosts included
# --------------------------------------------------------------------------

def as_grid(prob: Problem, q):
    return q.reshape(prob.ncomp, prob.ny, prob.nx)


def _pad(prob: Problem, g, axis):
    """Pad the (c, ny, nx) grid by one ghost layer along axis 2 (x) or 1 (y)."""
    n = g.shape[axis]
    first = np.take(g, [0], axis=axis)
    last = np.take(g, [n - 1], axis=axis)
    if prob.bc == BC_PERIODIC:
        lo, hi = last, first
    elif prob.bc == BC_TRANSMISSIVE:
        lo, hi = first, last
    else:  # inflow/outflow: only the x axis of a 1D grid has faces
        lo = np.full_like(first, prob.inflow)
        hi = last
    return np.concatenate([lo, g, hi], axis=axis)


def face_states(prob: Problem, q, axis):
    gp = _pad(prob, as_grid(prob, q), axis)
    n = gp.shape[axis]
    qL = np.take(gp, np.arange(0, n - 1), axis=axis)
    qR = np.take(gp, np.arange(1, n), axis=axis)
    return qL, qR


def face_flux(prob: Problem, qL, qR, axis):
    if prob.kind == EULER_2D:
        return euler_flux(qL, qR, prob.gamma, 1 if axis == 2 else 2)
    return burgers_flux(qL, qR)


def axes(prob: Problem):
    return (2,) if prob.kind == BURGERS_1D else (2, 1)


def lam(prob: Problem, axis):
    return prob.dt / prob.dx if axis == 2 else prob.dt / prob.dy


# --------------------------------------------------------------------------
# Residual  R_k(q) = q - q_prev + dt * div_h F(q)      (eq. hdm with BDF1)
# --------------------------------------------------------------------------

def residual(prob: Problem, q, q_prev):
    """Backward-Euler residual, component-major, same shape as q."""
    g = as_grid(prob, q)
    R = g - as_grid(prob, q_prev)
    for ax in axes(prob):
        qL, qR = face_states(prob, q, ax)
        F = face_flux(prob, qL, qR, ax)
        n = F.shape[ax]
        dF = np.take(F, np.arange(1, n), axis=ax) - np.take(F, np.arange(0, n - 1), axis=ax)
        R = R + lam(prob, ax) * dF
    return R.reshape(-1)


def cell_residual_norm(prob: Problem, q, q_prev):
    """Cellwise 2-norm of the residual over the components."""
    R = residual(prob, q, q_prev).reshape(prob.ncomp, prob.ncell)
    return np.sqrt(np.sum(R * R, axis=0))


# --------------------------------------------------------------------------
# Jacobian dR/dq, assembled from complex-step face-flux derivatives
# --------------------------------------------------------------------------

_CS_H = 1e-30


def face_flux_derivatives(prob: Problem, q, axis):
    """dF/dqL and dF/dqR at every face: arrays (c_out, c_in, *face_shape)."""
    qL, qR = face_states(prob, q, axis)
    c = prob.ncomp
    dL = np.empty((c, c) + qL.shape[1:])
    dR = np.empty((c, c) + qL.shape[1:])
    for k in range(c):
        e = np.zeros(qL.shape, dtype=complex)
        e[k] = 1j * _CS_H
        dL[:, k] = np.imag(face_flux(prob, qL + e, qR.astype(complex), axis)) / _CS_H
        dR[:, k] = np.imag(face_flux(prob, qL.astype(complex), qR + e, axis)) / _CS_H
    return dL, dR


def _face_sources(prob: Problem, axis):
    """For every face along ``axis``: cell index of the left and right state
    (-1 for a constant Dirichlet ghost) and the cell on each side that owns
    the face in its residual (-1 for none)."""
    nx, ny = prob.nx, prob.ny
    cell = np.arange(prob.ncell).reshape(ny, nx)
    if axis == 2:
        n = nx
        take = lambda i: cell[:, i]
    else:
        n = ny
        take = lambda i: cell[i, :]
    srcL, srcR, ownL, ownR = [], [], [], []
    for f in range(n + 1):
        if f == 0:
            if prob.bc == BC_PERIODIC:
                sl = take(n - 1)
            elif prob.bc == BC_TRANSMISSIVE:
                sl = take(0)
            else:
                sl = np.full_like(take(0), -1)
            ol = np.full_like(take(0), -1)
        else:
            sl = take(f - 1)
            ol = take(f - 1)
        if f == n:
            sr = take(0) if prob.bc == BC_PERIODIC else take(n - 1)
            orr = np.full_like(take(0), -1)
        else:
            sr = take(f)
            orr = take(f)
        srcL.append(sl); srcR.append(sr); ownL.append(ol); ownR.append(orr)
    # shape (n+1, other) -> match the face arrays, whose face axis is `axis`
    st = lambda lst: np.stack(lst, axis=(1 if axis == 2 else 0))
    return st(srcL), st(srcR), st(ownL), st(ownR)


def jacobian(prob: Problem, q, q_prev=None, cells=None) -> sp.csr_matrix:
    """Exact dR/dq (q_prev enters linearly with a constant, so it is unused).
    With ``cells`` only the rows of those cells' residuals are assembled (the
    others are left empty): the same entries, fewer of them."""
    c, nc = prob.ncomp, prob.ncell
    keep = None
    if cells is not None:
        keep = np.zeros(nc, dtype=bool)
        keep[np.asarray(cells, dtype=np.int64)] = True
    diag = np.arange(c * nc) if keep is None else dofs_of_cells(prob, np.flatnonzero(keep))
    rows, cols, vals = [diag], [diag], [np.ones(diag.size)]
    for ax in axes(prob):
        lx = lam(prob, ax)
        dL, dR = face_flux_derivatives(prob, q, ax)
        srcL, srcR, ownL, ownR = _face_sources(prob, ax)
        for own, sign in ((ownL, 1.0), (ownR, -1.0)):
            for src, d in ((srcL, dL), (srcR, dR)):
                ok = (own >= 0) & (src >= 0)
                if keep is not None:
                    ok &= keep[np.maximum(own, 0)]
                o = own[ok]
                s = src[ok]
                for a in range(c):
                    for b in range(c):
                        rows.append(a * nc + o)
                        cols.append(b * nc + s)
                        vals.append(sign * lx * d[a, b][ok])
    J = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(c * nc, c * nc))
    return J.tocsr()


# --------------------------------------------------------------------------
# Newton solves
# --------------------------------------------------------------------------

def newton_tol(q_prev) -> float:
    return NEWTON_RTOL * max(1.0, float(np.max(np.abs(q_prev))))


def hdm_step(prob: Problem, q_prev, tol=None, maxit=NEWTON_MAXIT):
    """Solve R_k(q) = 0 from the guess q_prev (eq. hdm).  Returns (q, iters)."""
    tol = newton_tol(q_prev) if tol is None else tol
    q = q_prev.copy()
    for it in range(maxit + 1):
        R = residual(prob, q, q_prev)
        if np.max(np.abs(R)) <= tol:
            return q, it
        if it == maxit:
            break
        J = jacobian(prob, q)
        q = q - spla.spsolve(J.tocsc(), R)
    raise NotConverged(f"HDM Newton: ||R||_inf = {np.max(np.abs(R)):.3e} > {tol:.3e}")


def dofs_of_cells(prob: Problem, cells):
    cells = np.asarray(cells, dtype=np.int64)
    return (np.arange(prob.ncomp)[:, None] * prob.ncell + cells[None, :]).reshape(-1)


def partial_hdm_solve(prob: Problem, u, q_prev, hat_cells, tol=None, maxit=NEWTON_MAXIT):
    """Solve the HDM residual restricted to the sampled cells (eq. partial_hdm2):
    hat-S^T R_k(hat-S v_hat + tilde-S v_tilde) = 0 for v_hat, every other
    entry of the full-size vector ``u`` held fixed.  Returns (u, iters)."""
    tol = newton_tol(q_prev) if tol is None else tol
    d = dofs_of_cells(prob, hat_cells)
    u = u.copy()
    for it in range(maxit + 1):
        R = residual(prob, u, q_prev)[d]
        if R.size == 0 or np.max(np.abs(R)) <= tol:
            return u, it
        if it == maxit:
            break
        J = jacobian(prob, u, cells=hat_cells)[d][:, d]
        u[d] = u[d] - spla.spsolve(J.tocsc(), R)
    raise NotConverged(f"partial HDM Newton: ||R||_inf = {np.max(np.abs(R)):.3e} > {tol:.3e}")
