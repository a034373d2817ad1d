"""Full-sensitivity Gauss-Newton on the reduced coordinates (oracle; test use only).

The subiterations of Sec. 2.3.2 alternate a partial HDM solve on the
sampled cells, with the neighbour ring held at psi + Phi y, and the gappy
fit of eq. red_coord.  Their fixed point y* satisfies
Phi_S^T (Phi_S y* - (v(y*) - psi_S)) = 0: the dependence of the sampled
solution v on y through the ring values is frozen.  This module minimises
the same misfit with that dependence kept,

    f(y) = 1/2 || r(y) ||^2,   r(y) = Phi_S y - (v(y) - psi_S),

where v(y) solves R_S(v; psi_T + Phi_T y) = 0 on the sampled set S with the
ring T held (eq. partial_hdm2).  Differentiating that equation,
dv/dy = -J_S^-1 J_T Phi_T (J_S, J_T the Jacobian's sampled rows restricted to
the sampled and ring columns), so the residual's Jacobian is

    A(y) = Phi_S + J_S^-1 J_T Phi_T   (m columns: m restricted linear solves)

and Gauss-Newton steps y <- y - A^+ r.  The first iterate is the paper's
first subiteration (the fit of the solve with the ring from gamma_{k-1});
the loop stops when ||dy||_2 < eps_y or after j_max iterations, as the
paper's.  Its stationarity condition A^T r = 0 differs from the paper's
Phi_S^T r = 0, so the two reach different points; the reconstruction,
filter and indicator then follow as in oracle.hybrid.  First-order scheme
(oracle.fv).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import fv
from .hybrid import HybridParams, fit, spatial_filter
from .sampling import indicator


def residual_jacobian(prob, u, q_prev, hd, td, Phi):
    """A = Phi_S + J_S^-1 J_T Phi_T at the state u (the converged partial
    solve), with its pieces."""
    cells = np.unique(hd % prob.ncell)
    J = fv.jacobian(prob, u, q_prev, cells=cells).tocsr()
    JS = J[hd][:, hd].tocsc()
    JT = J[hd][:, td]
    B = JT @ Phi[td] if td.size else np.zeros((hd.size, Phi.shape[1]))
    X = spla.spsolve(JS, B) if B.size else B
    X = np.asarray(X).reshape(hd.size, Phi.shape[1])
    return Phi[hd] + X, X


def gn_hybrid_step(prob, q_prev, Phi, psi, hat, tilde, params: HybridParams = None, record=None):
    """One hybrid snapshot with Gauss-Newton subiterations.  Returns dict(gamma,
    y, J, eps, rho, dy, newton, grad) with grad = A^T r at the last iterate."""
    params = params or HybridParams()
    hd = fv.dofs_of_cells(prob, hat)
    td = fv.dofs_of_cells(prob, tilde)
    u = q_prev.copy()
    newton, dy = [], []
    # first iterate: the paper's first subiteration
    u, its = fv.partial_hdm_solve(prob, u, q_prev, hat)
    newton.append(its)
    y = fit(Phi[hd], u[hd] - psi[hd], params.rcond_fit)
    J = 1
    grad = None
    for j in range(2, params.jmax + 1):
        u[td] = psi[td] + Phi[td] @ y
        u, its = fv.partial_hdm_solve(prob, u, q_prev, hat)
        newton.append(its)
        r = Phi[hd] @ y - (u[hd] - psi[hd])
        A, _ = residual_jacobian(prob, u, q_prev, hd, td, Phi)
        grad = A.T @ r
        step, *_ = np.linalg.lstsq(A, r, rcond=params.rcond_fit)
        y = y - step
        J = j
        dy.append(float(np.linalg.norm(step)))
        if record is not None:
            record.append({"y": y.copy(), "r": float(np.linalg.norm(r)), "grad": float(np.linalg.norm(grad))})
        if dy[-1] < params.eps_y:
            break
    # the state of the last iterate: the partial solve with the final ring
    u[td] = psi[td] + Phi[td] @ y
    u, its = fv.partial_hdm_solve(prob, u, q_prev, hat)
    newton.append(its)
    rho = psi + Phi @ y
    gamma = rho.copy()
    gamma[hd] = u[hd]
    gamma = spatial_filter(prob, gamma, q_prev, params)
    eps = indicator(prob, gamma, rho, params.floor_rel)
    return {"gamma": gamma, "y": y, "J": J, "eps": eps, "rho": rho, "dy": dy, "newton": newton, "grad": grad}
