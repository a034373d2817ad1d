"""Hybrid snapshot step (oracle; test use only).

Paper passages followed
-----------------------
* Hybrid approximation: affine-subspace values on the unsampled set and the
  restricted HDM on the sampled set (eq. hybrid: eq. rom_approx and
  eq. partial_hdm; eq. partial_hdm2).
* Gappy-POD reduced coordinates from the sampled rows (eq. red_coord).
* Subiterations between the partial HDM solve and the fit, started from the
  previous snapshot on the neighbour ring, stopped when the change of the
  reduced coordinates falls below eps_y or after j_max passes
  (Sec. 2.3.2, partial high-dimensional model; eps_y = 1e-4, j_max = 10).
* Reconstruction of the unsampled entries and the spatial filter
  (Alg. 1, hybrid branch).
* Residual-gated explicit Shapiro filters of increasing order, applied per
  coordinate direction with zeroth-order extrapolation at non-periodic
  boundaries (Sec. 2.3.4; eps_f = 1e-2, j_max^f = 10; filter orders 2, 4, 6
  as in both experiments).

Readings
--------
* The fit rows are the sampled set (no ODEIM points).
* The pseudo-inverse drops singular values of the gathered basis below
  rcond_fit times the largest (rcond_fit = 1e-8 by default, the square root
  of the double precision unit: below it a least-squares solution has no
  correct digits).
* The stopping test compares consecutive coordinates, so J >= 2.
* The Newton guess on the sampled set is the previous snapshot in the first
  subiteration and the previous subiteration's solution afterwards.
* Shapiro filter of order 2n: S_n = I - (-delta^2/4)^n, delta^2 the
  three-point second difference; in 2D x then y form one application.
* Gate: keep the filtered value where the cellwise residual 2-norm strictly
  decreases.  One filter order stops when no cell is kept, when the relative
  decrease of the l1 sum of the cell residual norms is below eps_f, or after
  j_max^f passes.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from workloads import BC_PERIODIC, BURGERS_1D, Problem

from . import fv
from .sampling import indicator, DEFAULT_FLOOR


@dataclasses.dataclass
class HybridParams:
    eps_y: float = 1e-4
    jmax: int = 10
    filter_orders: tuple = (1, 2, 3)      # n of S_n: filter orders 2, 4, 6
    eps_f: float = 1e-2
    jfmax: int = 10
    rcond_fit: float = 1e-8
    floor_rel: float = DEFAULT_FLOOR


# --------------------------------------------------------------------------
# Shapiro filters
# --------------------------------------------------------------------------

def shapiro_1d(prob: Problem, g, n, axis):
    """Apply S_n = I - (-delta^2/4)^n along one grid axis of a (c, ny, nx) array."""
    pad = [(0, 0)] * 3
    pad[axis] = (n, n)
    mode = "wrap" if prob.bc == BC_PERIODIC else "edge"
    w = np.pad(g, pad, mode=mode)
    for _ in range(n):
        m = w.shape[axis]
        lo = np.take(w, np.arange(0, m - 2), axis=axis)
        mid = np.take(w, np.arange(1, m - 1), axis=axis)
        hi = np.take(w, np.arange(2, m), axis=axis)
        w = -(lo - 2.0 * mid + hi) / 4.0
    return g - w


def shapiro(prob: Problem, q, n):
    g = fv.as_grid(prob, q)
    g = shapiro_1d(prob, g, n, 2)
    if prob.kind != BURGERS_1D:
        g = shapiro_1d(prob, g, n, 1)
    return g.reshape(-1)


def spatial_filter(prob: Problem, gamma, q_prev, params: HybridParams, log=None, masks=None, norms=None):
    """Residual-gated filter sequence.  Returns the filtered state.  If
    ``masks`` is a list, every applied pass appends (n, kept-cell mask); if
    ``norms`` is a list, every applied pass appends (n, r, rf), the cell
    residual norms its gate compared (a record only)."""
    c = prob.ncomp
    gamma = gamma.copy()
    for n in params.filter_orders:
        r = fv.cell_residual_norm(prob, gamma, q_prev)
        for it in range(1, params.jfmax + 1):
            gf = shapiro(prob, gamma, n)
            rf = fv.cell_residual_norm(prob, gf, q_prev)
            keep = rf < r
            nkeep = int(np.count_nonzero(keep))
            if log is not None:
                log.append((n, it, nkeep))
            if nkeep == 0:
                break
            km = np.tile(keep, c)
            gamma = np.where(km, gf, gamma)
            if masks is not None:
                masks.append((n, keep.copy()))
            if norms is not None:
                norms.append((n, r.copy(), rf.copy()))
            r_new = fv.cell_residual_norm(prob, gamma, q_prev)
            s_old = np.sum(r)
            s_new = np.sum(r_new)
            r = r_new
            if (s_old - s_new) / s_old < params.eps_f:
                break
    return gamma


# --------------------------------------------------------------------------
# The hybrid step
# --------------------------------------------------------------------------

def fit(Phi_rows, d, rcond):
    """Least-squares reduced coordinates with a truncated pseudo-inverse."""
    y, *_ = np.linalg.lstsq(Phi_rows, d, rcond=rcond)
    return y


def hybrid_step(prob: Problem, q_prev, Phi, psi, hat, tilde, params: HybridParams = None, norms=None,
                fit_points=None):
    """One hybrid snapshot gamma_k from gamma_{k-1} = q_prev.  With
    fit_points (entries of the state in sampled cells, e.g. ODEIM points:
    eq. red_coord's P) the fit uses those rows only.

    Returns dict(gamma, y, J, eps, rho, dy, newton, us, masks) where rho = psi + Phi y
    is the reconstruction, eps the indicator of the filtered snapshot, dy the
    norms ||y_j - y_{j-1}|| of the stopping test (j >= 2), us the
    state after each subiteration's Newton solve and masks the applied filter
    passes (the decisions the adjoint keeps frozen)."""
    params = params or HybridParams()
    hd = fv.dofs_of_cells(prob, hat)
    td = fv.dofs_of_cells(prob, tilde)
    fd = hd if fit_points is None else np.asarray(fit_points, dtype=np.int64)
    Phi_hat = Phi[fd]
    u = q_prev.copy()             # v_hat guess and v_tilde^(1) both from gamma_{k-1}
    y_old = None
    newton = []
    us = []
    dy = []
    J = 0
    for j in range(1, params.jmax + 1):
        u, its = fv.partial_hdm_solve(prob, u, q_prev, hat)
        newton.append(its)
        us.append(u.copy())
        y = fit(Phi_hat, u[fd] - psi[fd], params.rcond_fit)
        u[td] = psi[td] + Phi[td] @ y
        J = j
        if y_old is not None:
            dy.append(float(np.linalg.norm(y - y_old)))
            if dy[-1] < params.eps_y:
                break
        y_old = y
    rho = psi + Phi @ y
    gamma = rho.copy()
    gamma[hd] = u[hd]
    flog, masks = [], []
    gamma = spatial_filter(prob, gamma, q_prev, params, flog, masks, norms)
    eps = indicator(prob, gamma, rho, params.floor_rel)
    return {"gamma": gamma, "y": y, "J": J, "eps": eps, "rho": rho, "dy": dy,
            "newton": newton, "filter_log": flog, "us": us, "masks": masks}
