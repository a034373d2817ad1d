"""Why the basis update keeps its Gram in FP64 (CPU; numpy only).

The POD of eq. pod keeps every mode whose singular value is above 1e-8 of
the largest.  A Gram X^T X formed from FP32 data in FP32 arithmetic carries
an absolute error of about 2^-24 sigma_0^2 in every eigenvalue, so singular
values below about sqrt(2^-24) sigma_0 = 2.4e-4 sigma_0 are lost to rounding;
refinement inside the subspace that Gram spans cannot bring the lost
directions back.  The FP64 Gram keeps them to far below.  A planted
spectrum shows both.
"""
import numpy as np


def _planted(n=20000, w=24, seed=0):
    rng = np.random.default_rng(seed)
    sig = np.logspace(0, -8, w)
    U, _ = np.linalg.qr(rng.standard_normal((n, w)))
    V, _ = np.linalg.qr(rng.standard_normal((w, w)))
    return (U * sig) @ V.T, sig


def _singular_values_from_gram(G):
    lam = np.linalg.eigvalsh(G)[::-1]
    return np.sqrt(np.maximum(lam, 0.0))


def test_fp32_gram_loses_the_modes_the_pod_cut_keeps():
    X, sig = _planted()
    s64 = _singular_values_from_gram(X.T @ X)
    X32 = X.astype(np.float32)
    s32 = _singular_values_from_gram((X32.T @ X32).astype(np.float64))
    err64 = np.abs(s64 - sig) / sig
    err32 = np.abs(s32 - sig) / sig
    big = sig >= 1e-2
    lost = (sig <= 7e-5) & (sig >= 1e-6)
    assert lost.sum() >= 4
    # the leading modes: both fine
    assert np.all(err32[big] < 1e-3) and np.all(err64[big] < 1e-12)
    # below sqrt(2^-24) sigma_0: the FP32 Gram has no correct digit left,
    # the FP64 one still has five or more
    assert np.all(err32[lost] > 0.5), err32[lost]
    assert np.all(err64[lost] < 1e-5), err64[lost]
    # every one of those modes passes the POD cut of 1e-8 sigma_0
    assert np.all(sig[lost] > 1e-8 * sig[0])


def test_rounding_the_snapshots_alone_bounds_what_any_fp32_route_can_see():
    """Even with an exact (FP64) product, snapshots rounded to FP32 move each
    singular value by up to about 2^-24 sigma_0 (Weyl), so modes near 1e-8
    sigma_0 are out of reach of an FP32 copy of the window."""
    X, sig = _planted()
    X32 = X.astype(np.float32).astype(np.float64)
    s = np.linalg.svd(X32, compute_uv=False)
    pert = np.linalg.norm(X32 - X, 2)
    assert pert < 2.0 ** -24 * sig[0] * 4
    assert np.all(np.abs(s - sig) <= pert * (1 + 1e-6))
    tiny = sig < 1e-7
    assert np.any(np.abs(s - sig)[tiny] / sig[tiny] > 0.1)
