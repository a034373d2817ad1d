"""Pins of the oracle's ODEIM points (eq. odeim) against facts the
mathematics fixes (no GPU): QDEIM's pivots equal LAPACK's column-pivoted QR
of Phi^T, the published QDEIM bound on ||(P^T Phi)^-1||, the rank-one
eigenvalue bound that drives the oversampling (a true lower bound, exact for
m = 1), the monotone growth of sigma_min(P^T Phi), invariance of the points
under rotations of the basis, and exact recovery of coordinates in the
span by the fit over the points (eq. red_coord)."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import odeim


def orthonormal(rng, n, m, local=False):
    A = rng.standard_normal((n, m))
    if local:                                   # bumps: the shape of POD modes near moving waves
        x = np.linspace(0, 1, n)
        A = np.stack([np.exp(-((x - c) / 0.03) ** 2) * (1 + 0.1 * rng.standard_normal(n))
                      for c in rng.uniform(0.2, 0.8, m)], axis=1)
    Q, _ = np.linalg.qr(A)
    return Q


@pytest.mark.parametrize("n,m,local", [(60, 4, False), (200, 8, False), (300, 5, True)])
def test_qdeim_equals_lapack_pivoted_qr(n, m, local):
    Phi = orthonormal(np.random.default_rng(n + m), n, m, local)
    piv = sla.qr(Phi.T, pivoting=True, mode="r")[1]
    assert odeim.qdeim(Phi) == list(piv[:m])


@pytest.mark.parametrize("n,m,local", [(100, 3, False), (500, 6, True), (2000, 10, False)])
def test_qdeim_bound(n, m, local):
    """Drmac & Gugercin (2016): ||(P^T Phi)^-1||_2 <= sqrt(N - m + 1)
    sqrt(4^m + 6 m - 1) / 3 for orthonormal Phi."""
    Phi = orthonormal(np.random.default_rng(7 * n + m), n, m, local)
    P = odeim.qdeim(Phi)
    s = np.linalg.svd(Phi[P], compute_uv=False)
    assert 1.0 / s[-1] <= math.sqrt(n - m + 1) * math.sqrt(4 ** m + 6 * m - 1) / 3


@pytest.mark.parametrize("m", [1, 2, 4, 7])
def test_rank_one_bound_is_a_lower_bound(m):
    rng = np.random.default_rng(m)
    for _ in range(50):
        B = rng.standard_normal((m + 2, m))
        M = B.T @ B
        lam, U = np.linalg.eigh(M)
        rows = rng.standard_normal((20, m))
        gain = odeim.bound_gain(lam[0], lam[1] if m > 1 else None, U[:, 0], rows)
        for r, gval in zip(rows, gain):
            true = np.linalg.eigvalsh(M + np.outer(r, r))[0]
            assert gval >= -1e-14 and lam[0] + gval <= true + 1e-12 * max(1.0, true)
            if m == 1:
                assert abs(lam[0] + gval - true) <= 1e-12 * true


@pytest.mark.parametrize("n,m,n_p", [(200, 4, 8), (400, 6, 15), (120, 1, 4)])
def test_oversampling_raises_the_smallest_singular_value(n, m, n_p):
    Phi = orthonormal(np.random.default_rng(n * m), n, m, local=True)
    P = odeim.odeim(Phi, n_p)
    assert P[:m] == odeim.qdeim(Phi) and len(set(P)) == n_p
    smin = [np.linalg.svd(Phi[P[:k]], compute_uv=False)[-1] for k in range(m, n_p + 1)]
    assert all(b >= a - 1e-14 for a, b in zip(smin, smin[1:])), smin
    assert odeim.odeim(Phi, m) == odeim.qdeim(Phi)


@pytest.mark.parametrize("n,m,n_p", [(150, 4, 8), (300, 3, 9)])
def test_points_invariant_under_rotation_of_the_basis(n, m, n_p):
    rng = np.random.default_rng(n)
    Phi = orthonormal(rng, n, m, local=True)
    R, _ = np.linalg.qr(rng.standard_normal((m, m)))
    assert odeim.odeim(Phi @ R, n_p) == odeim.odeim(Phi, n_p)


def test_fit_over_the_points_recovers_coordinates_in_the_span():
    rng = np.random.default_rng(3)
    n, m = 250, 5
    Phi = orthonormal(rng, n, m, local=True)
    psi = rng.standard_normal(n)
    y = rng.standard_normal(m)
    v = psi + Phi @ y
    P = odeim.odeim(Phi, 2 * m)
    yf, *_ = np.linalg.lstsq(Phi[P], v[P] - psi[P], rcond=1e-8)
    assert np.max(np.abs(yf - y)) < 1e-12
    assert np.array_equal(odeim.cells_of([3, n + 3, 7], n), [3, 7])
