"""Oversampled empirical interpolation points (oracle; test use only).

eq. odeim: P_k = ODEIM_{n_p}(Phi_k), n_p > m points of the state vector whose
rows of Phi_k serve the least-squares fit of eq. red_coord, y = (P^T Phi)^+
P^T (v - psi).  The paper cites the method (Peherstorfer, Drmac and
Gugercin, 2020) without stating it; the reading implemented here:

* The first m points are those of QDEIM: the pivots of a column-pivoted QR
  of Phi^T.  Step j takes the row phi_i of Phi whose component orthogonal to
  the rows already taken has the largest norm, |phi_i|^2 - |Q^T phi_i|^2
  with Q an orthonormal basis of the taken rows (ties: lowest index).
* Each further point maximises a lower bound of the smallest eigenvalue of
  the sampled Gram after the rank-one update M + phi phi^T, M = Phi_P^T
  Phi_P: with M's two smallest eigenvalues l_1 <= l_2, the eigenvector u_1
  of l_1 and g = l_2 - l_1, the bound is
      l_1 + (g + |phi|^2 - sqrt((g + |phi|^2)^2 - 4 g (u_1^T phi)^2)) / 2
  (l_1 + (u_1^T phi)^2 when m = 1), so the row maximising the second term is
  taken (ties: lowest index; rows already taken are excluded).
* Points are entries of the state vector (a component of a cell); the
  sampled set holds whole cells, so the cells of the points join it.
* n_p = 2 m unless a caller states otherwise (the paper does not give n_p).
"""
from __future__ import annotations

import numpy as np


def qdeim(Phi, count=None):
    """The first ``count`` (default m) QDEIM points of the N x m basis."""
    n, m = Phi.shape
    count = m if count is None else count
    norms = np.einsum("ij,ij->i", Phi, Phi)
    Q = np.zeros((m, 0))
    taken = np.zeros(n, dtype=bool)
    pts = []
    for _ in range(count):
        proj = Phi @ Q
        score = norms - np.einsum("ij,ij->i", proj, proj)
        score[taken] = -np.inf
        p = int(np.argmax(score))           # first maximum: lowest index on ties
        pts.append(p)
        taken[p] = True
        v = Phi[p].copy()
        for _ in range(2):                  # Gram-Schmidt, twice
            v = v - Q @ (Q.T @ v)
        Q = np.column_stack([Q, v / np.linalg.norm(v)])
    return pts


def bound_gain(lam1, lam2, u1, rows):
    """The lower-bound gain of each candidate row (see the module text)."""
    a = rows @ u1
    b = np.einsum("ij,ij->i", rows, rows)
    if lam2 is None:
        return a * a
    g = lam2 - lam1
    s = g + b
    return 0.5 * (s - np.sqrt(np.maximum(s * s - 4.0 * g * a * a, 0.0)))


def odeim(Phi, n_p):
    """QDEIM's m points, then greedy oversampling to n_p points (in the
    order taken)."""
    n, m = Phi.shape
    if not m <= n_p <= n:
        raise ValueError("need m <= n_p <= N")
    pts = qdeim(Phi)
    taken = np.zeros(n, dtype=bool)
    taken[pts] = True
    while len(pts) < n_p:
        M = Phi[pts].T @ Phi[pts]
        lam, U = np.linalg.eigh(M)
        gain = bound_gain(lam[0], lam[1] if m > 1 else None, U[:, 0], Phi)
        gain[taken] = -np.inf
        p = int(np.argmax(gain))
        pts.append(p)
        taken[p] = True
    return pts


def cells_of(points, ncell):
    return np.unique(np.asarray(points, dtype=np.int64) % ncell).astype(np.int32)
