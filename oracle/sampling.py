"""Reconstruction-error indicator and sampling sets (oracle; test use only).

Paper passages followed
-----------------------
* Pointwise reconstruction error of the current snapshot against the affine
  subspace, Sec. 2.3.3 (relative reconstruction error).
* Descending ordering of the errors and the set G of the n_g largest,
  Sec. 2.3.3; the RRE rule for n_g, eq. rre.
* The sampled set as a union, its complement and the flux-stencil
  neighbours of it (Alg. 1, the set operations union / setdiff / Neighbors,
  and the sampling-matrix definitions of Sec. 2.3 with Fig. checkerboard).

Readings
--------
* The error is accumulated per cell (sum of squares over components); the
  paper indexes degrees of freedom but draws cells.
* Values below a floor are flushed to zero before ordering: a cell whose
  reconstruction error is at rounding level carries no information and its
  rank is not reproducible.  The floor is on the per-cell error norm,
  ``floor_rel * max(1, ||gamma||_inf)``; the default is 1e-14 (a few ulps
  of the state).
* Fixed-fraction mode (used by the workloads): n_g = min(ceil(f N_c),
  #{eps > 0}).  RRE mode: the smallest n_g with RRE(n_g) >= delta, with the
  sums of eq. rre taken exactly: every error is a dyadic rational
  M_i 2^(E_i), so all of them are written as integers over the smallest
  exponent present and the ratio test sum_top >= delta * sum is made in
  exact integer arithmetic (delta is itself a dyadic rational).  The count
  is then the paper's definition with no rounding and no dependence on a
  summation order.
* Ties in the ordering go to the lower cell index.
* No ODEIM points: the fit rows are the sampled set itself (the
  oversampling limit).  The sampled set is G dilated by a Chebyshev radius
  (2 cells by default, wrapping on periodic grids and clipped at walls).
* Neighbours are the face neighbours of the first-order flux stencil.
"""
from __future__ import annotations

import math

import numpy as np

from workloads import BC_PERIODIC, BURGERS_1D, Problem

RULE_FRACTION = 0
RULE_RRE = 1
DEFAULT_FLOOR = 1e-14


def indicator(prob: Problem, gamma, rho, floor_rel=DEFAULT_FLOOR):
    """eps_j = sum over components of (gamma - rho)^2 at cell j, where
    rho = psi + Phi y is the affine-subspace reconstruction; values whose
    cell norm is below the floor are set to 0."""
    d = (gamma - rho).reshape(prob.ncomp, prob.ncell)
    eps = np.sum(d * d, axis=0)
    floor = floor_rel * max(1.0, float(np.max(np.abs(gamma))))
    eps[eps < floor * floor] = 0.0
    return eps


def indicator_full(prob: Problem, gamma, Phi, psi, floor_rel=DEFAULT_FLOOR):
    """Indicator for a snapshot known everywhere: y = Phi^T (gamma - psi)
    (every row is a fit row and the basis is orthonormal)."""
    y = Phi.T @ (gamma - psi)
    return indicator(prob, gamma, psi + Phi @ y, floor_rel), y


def error_order(eps):
    """Cell indices by descending error, ties by ascending index."""
    return np.argsort(-eps, kind="stable")


def exact_dyadic(values):
    """Integers k_i and one exponent e with values_i = k_i 2^e exactly
    (non-negative doubles; e is the smallest binary exponent present)."""
    parts = []
    for v in values:
        if v <= 0.0:
            parts.append((0, 0))
            continue
        m, x = math.frexp(v)                 # v = m 2^x, 0.5 <= m < 1
        parts.append((int(m * (1 << 53)), x - 53))   # exact: v = M 2^(x - 53)
    e = min((x for M, x in parts if M > 0), default=0)
    return [M << (x - e) for M, x in parts], e


def count_g(eps, rule, fraction=0.0, delta=0.0):
    ncell = eps.size
    npos = int(np.count_nonzero(eps > 0))
    if rule == RULE_FRACTION:
        return min(int(math.ceil(fraction * ncell)), npos)
    if npos == 0:
        return 0
    # eq. rre: RRE(n) = sum_{top n} eps / sum eps; smallest n with RRE(n) >= delta
    k, _ = exact_dyadic(eps.tolist())
    total = sum(k)
    dm, de = math.frexp(float(delta))
    dnum, dexp = int(dm * (1 << 53)), de - 53    # delta = dnum 2^dexp exactly
    # S >= delta T  <=>  S 2^(-dexp) >= dnum T  (dexp < 0)  or  S >= dnum T 2^dexp
    rhs = dnum * total if dexp <= 0 else (dnum * total) << dexp
    sh = -dexp if dexp <= 0 else 0
    s = 0
    for g, i in enumerate(error_order(eps).tolist(), start=1):
        s += k[i]
        if (s << sh) >= rhs:
            return min(g, npos)
    return npos


def dilate(prob: Problem, mask, radius):
    """Chebyshev dilation of a cell mask by ``radius`` cells."""
    g = mask.reshape(prob.ny, prob.nx).copy()
    axes = (1,) if prob.kind == BURGERS_1D else (1, 0)
    for ax in axes:
        out = g.copy()
        n = g.shape[ax]
        for s in range(1, radius + 1):
            for sh in (s, -s):
                if prob.bc == BC_PERIODIC:
                    out |= np.roll(g, sh, axis=ax)
                elif n > s:
                    rolled = np.roll(g, sh, axis=ax)
                    idx = [slice(None)] * 2
                    idx[ax] = slice(0, sh) if sh > 0 else slice(n + sh, n)
                    rolled[tuple(idx)] = False
                    out |= rolled
        g = out
    return g.reshape(-1)


def neighbours(prob: Problem, mask):
    """Face neighbours of the cells in ``mask`` that are not themselves in it."""
    g = mask.reshape(prob.ny, prob.nx)
    nb = np.zeros_like(g)
    axes = (1,) if prob.kind == BURGERS_1D else (1, 0)
    for ax in axes:
        n = g.shape[ax]
        for sh in (1, -1):
            rolled = np.roll(g, sh, axis=ax)
            if prob.bc != BC_PERIODIC:
                idx = [slice(None)] * 2
                idx[ax] = slice(0, 1) if sh > 0 else slice(n - 1, n)
                rolled[tuple(idx)] = False
            nb |= rolled
    return (nb & ~g).reshape(-1)


def select(prob: Problem, eps, rule=RULE_FRACTION, fraction=0.1, delta=0.9, halo=2):
    """G (ordered), the sampled set and its neighbour ring (sorted cell lists)."""
    ng = count_g(eps, rule, fraction, delta)
    G = error_order(eps)[:ng]
    gmask = np.zeros(prob.ncell, dtype=bool)
    gmask[G] = True
    hat = dilate(prob, gmask, halo)
    tilde = neighbours(prob, hat)
    return {
        "G": G,
        "n_g": ng,
        "hat": np.flatnonzero(hat).astype(np.int32),
        "tilde": np.flatnonzero(tilde).astype(np.int32),
        "mask": hat,
    }
