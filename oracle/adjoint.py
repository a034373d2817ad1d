"""Discrete adjoint of the hybrid-snapshot trajectory (oracle; test use only).

The forward map u_0 -> u_T of Alg. 1 contains non-differentiable decisions:
the step schedule, the sampled sets, the subiteration count J, the filter
masks, the rank of the basis and of the fit.  The paper gives no adjoint of
its method; the one here (a reading of its Alg. 1 as a map of gamma_0)
differentiates the map with all of them frozen at their forward values, and with the bases Phi_k and reference states psi_k frozen as well
(they are functions of earlier snapshots; their derivatives are not taken).
With those frozen, each step is a smooth map of its input gamma_{k-1}:

* full step (eq. hdm): R(gamma_k; gamma_{k-1}) = 0, dR/dgamma_{k-1} = -I, so
  the tangent is J^{-1} d and the adjoint J^{-T} lambda;
* hybrid step (eq. hybrid, Sec. 2.3.2, Sec. 2.3.4): for j = 1..J the
  restricted solve R_S(v_j, t_j; p) = 0 on the sampled cells (t_1 = p on the
  neighbour ring), the fit y_j = A^+ (v_j - psi_S) with A = Phi on the sampled
  rows, t_{j+1} = psi_T + Phi_T y_j; then psi + Phi y_J on the unsampled
  cells, v_J on the sampled ones, and the frozen filter passes
  g <- M (S g) + (1 - M) g, a linear map.

Tangents (forward mode) and adjoints (reverse mode) are written separately so
that the dot-product test <T v, w> = <v, T^T w> checks the transposition.
The loss is L = 0.5 ||u_T - u_target||^2.

With ``psi_live`` the reference states are differentiated too: psi_k is the
mean of the w snapshots that eq. mean averages (for the basis update after
step k', the last w of its window, gamma_{k'-w+1} .. gamma_{k'}), a linear
map of those snapshots, so a hybrid step's adjoint with respect to its psi
(lambda_psi) returns lambda_psi / w to each of them.  The step is linear in
psi: the ring values t_{j+1} = psi_T + Phi_T y_j, the fit
y_j = A^+ (v_j - psi_S) and the reconstruction psi + Phi y_J off the sampled
cells.  Only the bases stay frozen.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from workloads import BC_PERIODIC, BURGERS_1D, Problem

from . import fv, pod, sampling
from .arom import AromParams, is_full_step, wants_update
from .hybrid import HybridParams, hybrid_step, shapiro


# --------------------------------------------------------------------------
# Forward with tape, and replay with frozen decisions
# --------------------------------------------------------------------------

def forward_with_tape(prob: Problem, q0, steps, p: AromParams, keep_norms=False):
    """Alg. 1 as in oracle.arom.run, recording every step's frozen data (with
    keep_norms also the residual norms each filter gate compared)."""
    gammas = [q0.copy()]
    basis = None
    samples = None
    tape = []
    for k in range(1, steps + 1):
        prev = gammas[-1]
        hybrid = (not is_full_step(k, p.w, p.z) and samples is not None and samples["hat"].size > 0
                  and basis is not None and basis[0].shape[1] > 0)
        eps = None
        if hybrid:
            norms = [] if keep_norms else None
            out = hybrid_step(prob, prev, basis[0], basis[1], samples["hat"], samples["tilde"], p.hybrid,
                              norms=norms)
            g = out["gamma"]
            eps = out["eps"]
            tape.append({"type": "hybrid", "hat": samples["hat"], "tilde": samples["tilde"],
                         "Phi": basis[0], "psi": basis[1], "psi_idx": basis[2], "J": out["J"],
                         "us": out["us"], "masks": out["masks"], "out": g, "norms": norms})
        else:
            g, _ = fv.hdm_step(prob, prev)
            tape.append({"type": "full", "out": g})
        gammas.append(g)
        samples = None
        if wants_update(k, p.w, p.z, steps):
            if k >= p.w and basis is not None and basis[0].shape[1] > 0:
                if eps is None:
                    eps, _ = sampling.indicator_full(prob, g, basis[0], basis[1], p.hybrid.floor_rel)
                samples = sampling.select(prob, eps, p.rule, p.fraction, p.delta, p.halo)
            window = gammas[k - p.w:k + 1] if k >= p.w else gammas[0:k + 1]
            b = pod.pod(window, p.w, p.m, p.tau_pod)
            # psi_new is the mean of the window's last w snapshots
            basis = (b["Phi"], b["psi_new"], list(range(k - p.w + 1, k + 1)))
    return gammas[-1], tape


def replay_hybrid(prob: Problem, q_prev, st, params: HybridParams, states=False):
    """The hybrid step with J, the sets, the basis and the filter masks frozen.
    With ``states`` also the state after each subiteration's Newton solve."""
    hd = fv.dofs_of_cells(prob, st["hat"])
    td = fv.dofs_of_cells(prob, st["tilde"])
    Phi, psi = st["Phi"], st["psi"]
    u = q_prev.copy()
    us = []
    for _ in range(st["J"]):
        u, _ = fv.partial_hdm_solve(prob, u, q_prev, st["hat"])
        us.append(u.copy())
        y, *_ = np.linalg.lstsq(Phi[hd], u[hd] - psi[hd], rcond=params.rcond_fit)
        u[td] = psi[td] + Phi[td] @ y
    g = psi + Phi @ y
    g[hd] = u[hd]
    for n, keep in st["masks"]:
        g = np.where(np.tile(keep, prob.ncomp), shapiro(prob, g, n), g)
    return (g, us) if states else g


def replay(prob: Problem, q0, tape, params: HybridParams, psi_live=False):
    """The frozen trajectory from q0.  With psi_live each hybrid step's psi is
    the plain mean of its snapshots of this run (the map whose derivative
    gradient(..., psi_live=True) takes); otherwise the recorded psi."""
    q = q0.copy()
    states = [q]
    for st in tape:
        if st["type"] == "full":
            q, _ = fv.hdm_step(prob, q)
        else:
            if psi_live:
                st = dict(st, psi=sum(states[j] for j in st["psi_idx"]) / len(st["psi_idx"]))
            q = replay_hybrid(prob, q, st, params)
        states.append(q)
    return q


# --------------------------------------------------------------------------
# Linear pieces
# --------------------------------------------------------------------------

def _stencil_weights(n):
    """Weights of (-delta^2/4)^n on a line (length 2n+1)."""
    e = np.zeros(4 * n + 1)
    e[2 * n] = 1.0
    w = e
    for _ in range(n):
        w = -(w[:-2] - 2.0 * w[1:-1] + w[2:]) / 4.0
    return w[::-1]                  # correlation weights for offsets -n..n


def shapiro_1d_T(prob: Problem, h, n, axis):
    """Transpose of the 1D filter along ``axis`` of a (c, ny, nx) array.

    The filter is S = I - K E with E the extension by n cells (periodic wrap or
    repetition of the boundary value) and K the (2n+1)-point stencil on the
    extended line; so S^T = I - E^T K^T."""
    w = _stencil_weights(n)
    L = h.shape[axis]
    shape = list(h.shape)
    shape[axis] = L + 2 * n
    full = np.zeros(shape)
    for k in range(2 * n + 1):          # K^T: scatter h back onto the extended line
        sl = [slice(None)] * 3
        sl[axis] = slice(k, k + L)
        full[tuple(sl)] += w[k] * h
    take = lambda a, b: np.take(full, np.arange(a, b), axis=axis)
    out = take(n, n + L).copy()
    if prob.bc == BC_PERIODIC:          # E^T: wrapped margins return to their cells
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(L - n, L)
        hi[axis] = slice(0, n)
        out[tuple(lo)] += take(0, n)
        out[tuple(hi)] += take(n + L, L + 2 * n)
    else:                               # E^T: repeated boundary values return to it
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, 1)
        hi[axis] = slice(L - 1, L)
        out[tuple(lo)] += np.sum(take(0, n), axis=axis, keepdims=True)
        out[tuple(hi)] += np.sum(take(n + L, L + 2 * n), axis=axis, keepdims=True)
    return h - out


def shapiro_T(prob: Problem, q, n):
    """Transpose of the 2D filter S = S_y S_x (S^T = S_x^T S_y^T)."""
    g = fv.as_grid(prob, q)
    if prob.kind != BURGERS_1D:
        g = shapiro_1d_T(prob, g, n, 1)
    g = shapiro_1d_T(prob, g, n, 2)
    return g.reshape(-1)


def _split_jacobian(prob: Problem, u, hat, tilde):
    J = fv.jacobian(prob, u)
    hd = fv.dofs_of_cells(prob, hat)
    td = fv.dofs_of_cells(prob, tilde)
    Jh = J[hd][:, hd].tocsc()
    Jt = J[hd][:, td].tocsc() if td.size else None
    return Jh, Jt, hd, td


def _pinv(st, hd, params):
    return np.linalg.pinv(st["Phi"][hd], rcond=params.rcond_fit)


# --------------------------------------------------------------------------
# Tangents
# --------------------------------------------------------------------------

def full_step_tangent(prob: Problem, q_out, d):
    return spla.spsolve(fv.jacobian(prob, q_out).tocsc(), d)


def hybrid_step_tangent(prob: Problem, st, d, params: HybridParams):
    Phi = st["Phi"]
    hd = fv.dofs_of_cells(prob, st["hat"])
    td = fv.dofs_of_cells(prob, st["tilde"])
    Ap = _pinv(st, hd, params)
    dt = d[td]
    for j in range(st["J"]):
        Jh, Jt, _, _ = _split_jacobian(prob, st["us"][j], st["hat"], st["tilde"])
        rhs = d[hd] - (Jt @ dt if Jt is not None else 0.0)
        dv = spla.spsolve(Jh, rhs)
        dy = Ap @ dv
        dt = Phi[td] @ dy
    g = Phi @ dy
    g[hd] = dv
    for n, keep in st["masks"]:
        g = np.where(np.tile(keep, prob.ncomp), shapiro(prob, g, n), g)
    return g


# --------------------------------------------------------------------------
# Adjoints
# --------------------------------------------------------------------------

def full_step_adjoint(prob: Problem, q_out, lam):
    return spla.spsolve(fv.jacobian(prob, q_out).T.tocsc(), lam)


def hybrid_step_adjoint(prob: Problem, st, lam, params: HybridParams):
    Phi = st["Phi"]
    N = prob.n
    hd = fv.dofs_of_cells(prob, st["hat"])
    td = fv.dofs_of_cells(prob, st["tilde"])
    Ap = _pinv(st, hd, params)
    g = lam.copy()
    for n, keep in reversed(st["masks"]):          # pass map P = D S + (I - D)
        km = np.tile(keep, prob.ncomp)
        g = shapiro_T(prob, np.where(km, g, 0.0), n) + np.where(km, 0.0, g)
    breve = np.ones(N, bool)
    breve[hd] = False
    ybar = Phi[breve].T @ g[breve]
    vbar = g[hd].copy()
    tbar_next = np.zeros(td.size)
    pbar = np.zeros(N)
    for j in reversed(range(st["J"])):
        ybar_j = (ybar if j == st["J"] - 1 else 0.0) + Phi[td].T @ tbar_next
        vbar_j = (vbar if j == st["J"] - 1 else 0.0) + Ap.T @ ybar_j
        Jh, Jt, _, _ = _split_jacobian(prob, st["us"][j], st["hat"], st["tilde"])
        mu = spla.spsolve(Jh.T.tocsc(), vbar_j)
        pbar[hd] += mu
        tbar_next = -(Jt.T @ mu) if Jt is not None else np.zeros(0)
    pbar[td] += tbar_next
    return pbar


def hybrid_step_tangent_psi(prob: Problem, st, dpsi, params: HybridParams):
    """Derivative of the frozen hybrid step's output with respect to its psi
    (gamma_{k-1} fixed), applied to dpsi."""
    Phi = st["Phi"]
    hd = fv.dofs_of_cells(prob, st["hat"])
    td = fv.dofs_of_cells(prob, st["tilde"])
    Ap = _pinv(st, hd, params)
    dt = np.zeros(td.size)                    # t_1 = gamma_{k-1} on the ring: no psi
    for j in range(st["J"]):
        Jh, Jt, _, _ = _split_jacobian(prob, st["us"][j], st["hat"], st["tilde"])
        dv = spla.spsolve(Jh, -(Jt @ dt)) if Jt is not None else np.zeros(hd.size)
        dy = Ap @ (dv - dpsi[hd])
        dt = dpsi[td] + Phi[td] @ dy
    g = dpsi + Phi @ dy
    g[hd] = dv
    for n, keep in st["masks"]:
        g = np.where(np.tile(keep, prob.ncomp), shapiro(prob, g, n), g)
    return g


def hybrid_step_adjoint_psi(prob: Problem, st, lam, params: HybridParams):
    """(gamma_{k-1} adjoint, psi adjoint) of the frozen hybrid step: the
    transpose of hybrid_step_tangent and of hybrid_step_tangent_psi."""
    Phi = st["Phi"]
    N = prob.n
    hd = fv.dofs_of_cells(prob, st["hat"])
    td = fv.dofs_of_cells(prob, st["tilde"])
    Ap = _pinv(st, hd, params)
    g = lam.copy()
    for n, keep in reversed(st["masks"]):
        km = np.tile(keep, prob.ncomp)
        g = shapiro_T(prob, np.where(km, g, 0.0), n) + np.where(km, 0.0, g)
    breve = np.ones(N, bool)
    breve[hd] = False
    psibar = np.where(breve, g, 0.0)            # reconstruction psi + Phi y off the sampled cells
    ybar = Phi[breve].T @ g[breve]
    vbar = g[hd].copy()
    tbar_next = np.zeros(td.size)
    pbar = np.zeros(N)
    for j in reversed(range(st["J"])):
        if j < st["J"] - 1:
            psibar[td] += tbar_next               # t_{j+1} = psi_T + Phi_T y_j
        ybar_j = (ybar if j == st["J"] - 1 else 0.0) + Phi[td].T @ tbar_next
        w_j = Ap.T @ ybar_j                       # y_j = A^+ (v_j - psi_S)
        psibar[hd] -= w_j
        vbar_j = (vbar if j == st["J"] - 1 else 0.0) + w_j
        Jh, Jt, _, _ = _split_jacobian(prob, st["us"][j], st["hat"], st["tilde"])
        mu = spla.spsolve(Jh.T.tocsc(), vbar_j)
        pbar[hd] += mu
        tbar_next = -(Jt.T @ mu) if Jt is not None else np.zeros(0)
    pbar[td] += tbar_next                         # t_1 = gamma_{k-1} on the ring
    return pbar, psibar


def step_adjoint(prob: Problem, st, lam, params: HybridParams):
    if st["type"] == "full":
        return full_step_adjoint(prob, st["out"], lam)
    return hybrid_step_adjoint(prob, st, lam, params)


def step_tangent(prob: Problem, st, d, params: HybridParams):
    if st["type"] == "full":
        return full_step_tangent(prob, st["out"], d)
    return hybrid_step_tangent(prob, st, d, params)


def gradient(prob: Problem, tape, qT, target, params: HybridParams, psi_live=False):
    """dL/du_0 for L = 0.5 ||u_T - u_target||^2 through the frozen trajectory
    (with psi_live also through each hybrid step's reference state)."""
    return backward(prob, tape, qT - target, params, psi_live)


def backward(prob: Problem, tape, lam_T, params: HybridParams, psi_live=False):
    """(d gamma_T / d gamma_0)^T lam_T through the frozen trajectory.  With
    psi_live, the psi adjoint of the hybrid step that ends in gamma_k is held
    until the backward pass reaches each snapshot its psi averages, and
    added there with weight 1/w."""
    lam = lam_T.copy()
    pending = {}                                  # snapshot index -> accumulated psi contributions
    for k in range(len(tape), 0, -1):
        if k in pending:
            lam = lam + pending.pop(k)
        st = tape[k - 1]
        if st["type"] == "full" or not psi_live:
            lam = step_adjoint(prob, st, lam, params)
            continue
        lam, psibar = hybrid_step_adjoint_psi(prob, st, lam, params)
        share = psibar / len(st["psi_idx"])
        for j in st["psi_idx"]:
            pending[j] = pending[j] + share if j in pending else share.copy()
    if 0 in pending:
        lam = lam + pending.pop(0)
    return lam


def loss(qT, target):
    d = qT - target
    return 0.5 * float(d @ d)
