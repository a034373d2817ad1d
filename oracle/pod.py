"""Window mean and POD basis (oracle; test use only).

Paper passages followed
-----------------------
* The reference state is the mean of the previous w snapshots (eq. mean);
  the first one is the mean of snapshots 0..w-1 (Alg. 1, the offset set at
  k = w-1).
* The basis is POD_m of the window deviations from the *lagged* reference
  state: the thin SVD of the N x w snapshot matrix and its first m left
  singular vectors (eq. pod; Alg. 1, basis update).

Readings
--------
* Snapshot list convention: ``snaps`` holds gamma_{k-w}, ..., gamma_k
  (w + 1 entries) or, at the first update, gamma_0, ..., gamma_{w-1}
  (w entries).  The centring state is the mean of the first w entries and
  the new reference state the mean of the last w entries; with w entries
  both are the same mean, as Alg. 1 prescribes at k = w - 1.
* Means: the exact sum of the w snapshots, rounded once to double (the
  correctly rounded sum), divided by w.  A plain floating-point sum would
  make the last bit of every entry depend on the summation order; entries of
  the window deviations X are then equal to the bit in any implementation
  that rounds the sum correctly, and the POD of two implementations differs
  only by their own SVD rounding (a one-ulp difference of the centring
  state is a rank-one change of X of norm ~ulp sqrt(N w), which on large
  grids exceeds the smallest singular values that are still resolvable).
* Rank truncation: modes with sigma_i <= tau_pod sigma_1 are dropped
  (m_eff <= m); tau_pod = 1e-8 by default.  POD_m keeps m vectors, but a
  window of smooth, slowly moving snapshots has singular values that fall
  to the rounding level (eps sigma_1) well before m; their vectors are
  rounding noise, not reproducible by any two correct SVDs.  Modes above
  1e-8 sigma_1 are determined to about eps sigma_1 / gap; the dropped ones
  carry less than 1e-16 of the window energy.  (With 1e-4 instead, the
  1D Burgers (1024 cells) and 2D Burgers runs keep 4 and 18 modes instead of 10 and 32 and their
  error against the full model is 1.5 to 3 times larger.)
* Sign: each right singular vector has its largest-magnitude entry
  positive (lowest index on ties); the left vector takes the same sign.
"""
from __future__ import annotations

import math

import numpy as np

DEFAULT_TAU = 1e-8


def window_mean(snaps):
    """(1/w) * sum of the snapshots, the sum correctly rounded entry by entry."""
    rows = np.stack(snaps, axis=1).tolist()
    return np.array([math.fsum(r) for r in rows], dtype=np.float64) / len(snaps)


def centring_and_new_mean(snaps, w):
    if len(snaps) not in (w, w + 1):
        raise ValueError("window must hold w or w+1 snapshots")
    return window_mean(snaps[:w]), window_mean(snaps[-w:])


def pod(snaps, w, m, tau=DEFAULT_TAU):
    """Returns dict(Phi (N x m_eff), sigma (w), m_eff, psi_centre, psi_new, V)."""
    centre, psi_new = centring_and_new_mean(snaps, w)
    X = np.stack([s - centre for s in snaps[-w:]], axis=1)
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    m_eff = int(np.count_nonzero(s[:m] > tau * s[0])) if s[0] > 0 else 0
    Phi = U[:, :m_eff].copy()
    V = Vt[:m_eff].T.copy()
    for i in range(m_eff):
        j = int(np.argmax(np.abs(V[:, i])))
        if V[j, i] < 0:
            V[:, i] = -V[:, i]
            Phi[:, i] = -Phi[:, i]
    return {"Phi": Phi, "sigma": s, "m_eff": m_eff, "psi_centre": centre,
            "psi_new": psi_new, "V": V, "X": X}
