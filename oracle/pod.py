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
* Means are plain sequential sums divided by w.
* Rank truncation: modes with sigma_i <= tau_pod sigma_1 are dropped
  (m_eff <= m); tau_pod = 1e-4 by default.  Trailing singular vectors of a
  window of smooth, slowly moving snapshots are rounding noise and not
  reproducible; the dropped modes carry less than 1e-8 of the window energy.
* Sign: each right singular vector has its largest-magnitude entry
  positive (lowest index on ties); the left vector takes the same sign.
"""
from __future__ import annotations

import numpy as np

DEFAULT_TAU = 1e-4


def window_mean(snaps):
    acc = np.zeros_like(snaps[0])
    for s in snaps:
        acc = acc + s
    return acc / len(snaps)


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
