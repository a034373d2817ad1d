"""Algorithm 1 and its hybrid step on the paper's own HDM (oracle; test use only).

The same method as oracle.hybrid / oracle.arom, with the full-order model of
Sec. 3.1 (oracle.paper_hdm: MUSCL + minmod, Roe, BDF2):

* Every step's residual is the BDF2 residual of eq. hdm with q_{k-2} (BDF1 at
  k = 1), on full, partial (eq. partial_hdm2) and filter-gate evaluations
  alike, for full and hybrid steps.
* The neighbour ring S~ is every cell the residual of the sampled cells
  reads outside the sampled set: the reconstruction stencil reaches two
  cells along each axis, so S~ holds the cells within two cells, along an
  axis, of a sampled cell (Sec. 2.3.2's partial HDM with this scheme).
* The partial solve is Newton on the restricted residual with the oracle's
  colour-grouped finite-difference Jacobian (rows and columns of the sampled
  cells), to ||R||_inf <= 1e-13 max(1, |q_{k-1}|_inf).
* Selection (dilation by the halo), the indicator, the fit, the filters and
  the POD are those of oracle.sampling, oracle.hybrid and oracle.pod; the
  Shapiro filters extrapolate by zeroth order at the (non-periodic)
  boundaries, as there.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from workloads import BC_TRANSMISSIVE, EULER_2D, Problem

from . import odeim as od
from . import paper_hdm as ph
from . import pod, sampling
from .arom import AromParams, is_full_step, wants_update
from .hybrid import HybridParams, fit, shapiro

RTOL = 1e-13


class NotConverged(RuntimeError):
    pass


def view(prob: ph.PaperProblem) -> Problem:
    """The mesh as the selection, indicator and filter routines see it."""
    return Problem(kind=EULER_2D, nx=prob.nx, ny=prob.ny, bc=BC_TRANSMISSIVE, dx=prob.dx, dy=prob.dy,
                   dt=prob.dt, gamma=prob.gamma, inflow=0.0)


def dofs(prob: ph.PaperProblem, cells):
    cells = np.asarray(cells, dtype=np.int64)
    return (np.arange(4)[:, None] * prob.ncell + cells[None, :]).reshape(-1)


def ring(prob: ph.PaperProblem, hat_mask):
    """Cells within two cells along an axis of a sampled cell, not sampled."""
    g = hat_mask.reshape(prob.ny, prob.nx)
    out = np.zeros_like(g)
    axes = (1,) if prob.ny == 1 else (1, 0)
    for ax in axes:
        n = g.shape[ax]
        for s in (1, 2, -1, -2):
            if n <= abs(s):
                continue
            rolled = np.roll(g, s, axis=ax)
            idx = [slice(None)] * 2
            idx[ax] = slice(0, s) if s > 0 else slice(n + s, n)
            rolled[tuple(idx)] = False
            out |= rolled
    return (out & ~g).reshape(-1)


def cell_residual_norm(prob: ph.PaperProblem, q, q1, q2):
    R = ph.residual(prob, q, q1, q2).reshape(4, prob.ncell)
    return np.sqrt(np.sum(R * R, axis=0))


def partial_solve(prob: ph.PaperProblem, u, q1, q2, hat, maxit=30):
    """Newton on the residual rows of the sampled cells for their entries,
    every other entry of u held (eq. partial_hdm2).  Returns (u, iterations)."""
    tol = RTOL * max(1.0, float(np.max(np.abs(q1))))
    d = dofs(prob, hat)
    u = u.copy()
    for it in range(maxit + 1):
        R = ph.residual(prob, u, q1, q2)[d]
        if R.size == 0 or np.max(np.abs(R)) <= tol:
            return u, it
        if it == maxit:
            break
        J = ph.fd_jacobian(prob, u, q1, q2)[d][:, d]
        u[d] = u[d] - spla.spsolve(J.tocsc(), R)
    raise NotConverged(f"partial Newton: ||R||_inf = {np.max(np.abs(R)):.3e} > {tol:.3e}")


def spatial_filter(prob: ph.PaperProblem, gamma, q1, q2, params: HybridParams, log=None, masks=None):
    """The residual-gated filter sequence of Sec. 2.3.4 with this scheme's
    cell residual norms (the loop of oracle.hybrid.spatial_filter)."""
    v = view(prob)
    gamma = gamma.copy()
    for n in params.filter_orders:
        r = cell_residual_norm(prob, gamma, q1, q2)
        for it in range(1, params.jfmax + 1):
            gf = shapiro(v, gamma, n)
            rf = cell_residual_norm(prob, gf, q1, q2)
            keep = rf < r
            nkeep = int(np.count_nonzero(keep))
            if log is not None:
                log.append((n, it, nkeep))
            if nkeep == 0:
                break
            gamma = np.where(np.tile(keep, 4), gf, gamma)
            if masks is not None:
                masks.append((n, keep.copy()))
            r_new = cell_residual_norm(prob, gamma, q1, q2)
            s_old, s_new = np.sum(r), np.sum(r_new)
            r = r_new
            if (s_old - s_new) / s_old < params.eps_f:
                break
    return gamma


def hybrid_step(prob: ph.PaperProblem, q1, q2, Phi, psi, hat, params: HybridParams = None, fit_points=None):
    """One hybrid snapshot gamma_k from gamma_{k-1} = q1 (and q_{k-2} = q2).
    With fit_points (entries of the state, their cells sampled) the fit of
    eq. red_coord uses those rows only; otherwise every entry of the sampled
    cells."""
    params = params or HybridParams()
    hat = np.asarray(hat)
    mask = np.zeros(prob.ncell, dtype=bool)
    mask[hat] = True
    tilde = np.flatnonzero(ring(prob, mask))
    hd, td = dofs(prob, hat), dofs(prob, tilde)
    fd = hd if fit_points is None else np.asarray(fit_points, dtype=np.int64)
    Phi_fit = Phi[fd]
    u = q1.copy()
    y_old, newton, dy, J = None, [], [], 0
    for j in range(1, params.jmax + 1):
        u, its = partial_solve(prob, u, q1, q2, hat)
        newton.append(its)
        y = fit(Phi_fit, u[fd] - psi[fd], params.rcond_fit)
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
    gamma = spatial_filter(prob, gamma, q1, q2, params, flog, masks)
    eps = sampling.indicator(view(prob), gamma, rho, params.floor_rel)
    return {"gamma": gamma, "y": y, "J": J, "eps": eps, "rho": rho, "dy": dy, "newton": newton,
            "filter_log": flog, "masks": masks, "l": int(tilde.size)}


def run(prob: ph.PaperProblem, q0, steps, p: AromParams, keep_all=False, on_step=None, odeim_factor=0):
    """Alg. 1 with this scheme (the schedule, updates and fallback of
    oracle.arom.run).  With odeim_factor > 0 the sampled set of each hybrid
    step also holds the cells of n_p = odeim_factor m_eff ODEIM points of its
    basis (eq. odeim; Alg. 1: P_{k+1} from Phi_{k+1}, then the union with G),
    and the fit uses those points only (eq. red_coord).  Returns dict(q,
    records, gammas)."""
    v = view(prob)
    gammas = [q0.copy()]
    basis, samples, records = None, None, []
    for k in range(1, steps + 1):
        rec = {"k": k}
        q1 = gammas[-1]
        q2 = gammas[-2] if k >= 2 else None
        hybrid_ok = (not is_full_step(k, p.w, p.z) and samples is not None and samples["hat"].size > 0
                     and basis is not None and basis[0].shape[1] > 0)
        eps = None
        if hybrid_ok:
            try:
                out = hybrid_step(prob, q1, q2, basis[0], basis[1], samples["hat"], p.hybrid,
                                  fit_points=samples.get("points"))
                g, eps = out["gamma"], out["eps"]
                rec.update(type="hybrid", n_s=int(samples["hat"].size), l=out["l"], J=out["J"],
                           newton=out["newton"], n_p=len(samples.get("points", ())))
            except NotConverged:
                hybrid_ok = False
        if not hybrid_ok:
            g, its = ph.hdm_step(prob, q1, q2, rtol=RTOL)
            rec.update(type="full", n_s=prob.ncell, newton=[its])
        gammas.append(g)
        if not keep_all and len(gammas) > p.w + 2:
            gammas[-(p.w + 3)] = None
        samples = None
        if wants_update(k, p.w, p.z, steps):
            if k >= p.w and basis is not None and basis[0].shape[1] > 0:
                if eps is None:
                    eps, _ = sampling.indicator_full(v, g, basis[0], basis[1], p.hybrid.floor_rel)
                samples = sampling.select(v, eps, p.rule, p.fraction, p.delta, p.halo)
                rec["n_g"] = samples["n_g"]
            window = gammas[k - p.w:k + 1] if k >= p.w else gammas[0:k + 1]
            b = pod.pod(window, p.w, p.m, p.tau_pod)
            basis = (b["Phi"], b["psi_new"])
            rec["m_eff"] = b["m_eff"]
            if odeim_factor and samples is not None and b["m_eff"] > 0:
                pts = od.odeim(b["Phi"], min(odeim_factor * b["m_eff"], prob.n))
                hat = np.union1d(samples["hat"], od.cells_of(pts, prob.ncell)).astype(np.int32)
                samples = {**samples, "hat": hat, "points": pts}
        records.append(rec)
        if on_step is not None:
            on_step(k, g, rec)
    return {"q": gammas[-1], "records": records, "gammas": gammas if keep_all else None}
