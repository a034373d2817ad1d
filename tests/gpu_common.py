"""Shared helpers for the GPU parity tests (imported only by tests)."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def ctx_for(prob, m_max=64, w_max=64, **kw):
    import paper_2301_01718_amd as hs
    return hs.Context(prob, m_max=m_max, w_max=w_max, **kw)


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


# small cases spanning several blocks and a ragged tail
CASES = {
    "burgers1d": (W.WORKLOADS["burgers1d_1k"], 1000, 1),
    "burgers2d": (W.WORKLOADS["burgers2d_1024"], 67, 53),
    "euler2d": (W.WORKLOADS["euler2d_512"], 45, 37),
}


def case(name, seed=0):
    wl, nx, ny = CASES[name]
    wl = wl.resized(nx, ny)
    prob, q0 = W.make(wl, seed)
    return wl, prob, q0


def print_case(*args):
    print("CASE", *args, flush=True)


def indicator_close(eg, eo, gamma, floor_rel=1e-14, tol=1e-13, cell_tol=None):
    """Compare two indicators through the error norms sqrt(eps) (eps is the
    square of a difference of nearly equal states; its reproducible part is
    the norm).  sqrt(eps) = |gamma - rho| per cell, so it inherits the state's
    parity: norm-wise within tol ||gamma||_2 (the state's bar), and cell by
    cell within cell_tol max(1, |gamma|_inf) (default tol; after a hybrid step
    the callers pass 100 tol: a restricted Newton root is only fixed to its
    tolerance, and the fit spreads that over the reconstruction by the
    gathered basis' condition number).  A cell may flip between flushed and
    kept only within 1 % of the floor."""
    scale = max(1.0, float(np.max(np.abs(gamma))))
    fl = floor_rel * scale
    a, b = np.sqrt(eg), np.sqrt(eo)
    near_floor = (np.minimum(np.where(a > 0, a, np.inf), np.where(b > 0, b, np.inf)) < 1.01 * fl)
    diff = np.where(near_floor, 0.0, np.abs(a - b))
    cell_tol = tol if cell_tol is None else cell_tol
    ok = np.linalg.norm(diff) <= tol * np.linalg.norm(gamma) and np.all(diff <= cell_tol * scale)
    return bool(ok), float(np.max(diff) / scale)


def fit_tols(fit_cond, tol=1e-12, cell_tol=1e-10):
    """The indicator's tolerances after a hybrid step whose gathered basis
    has condition number (bound) fit_cond: sqrt(eps) on the sampled cells is
    the fit's misfit |v - psi - Phi y|, and two correct least-squares
    solutions differ by about kappa^2 eps relative (their sensitivity to
    rounding), so the bars grow with 10 kappa^2 eps once that exceeds them."""
    k2e = 10.0 * float(fit_cond) ** 2 * 2.2e-16
    return max(tol, k2e), max(cell_tol, 100.0 * k2e)


def state_tol(fit_cond, tol=1e-12):
    """The state bar of a hybrid step whose gathered basis has condition
    number (bound) fit_cond: the unsampled cells are psi + Phi y, and for a
    least-squares fit with a small residual (the misfit on the sampled cells
    is O(sqrt(eps)) relative) first-order perturbation theory bounds the
    relative difference of two correct solutions y by about kappa eps, so the
    bar grows with 10 kappa eps once that exceeds tol."""
    return max(tol, 10.0 * float(fit_cond) * 2.2e-16)


def projector_tol(sigma, me, c=100.0):
    """Bound on ||P_gpu X - P_oracle X|| / ||X|| for the orthogonal projectors
    onto two rank-me POD subspaces of the same window.  Both SVDs are exact for
    X + E with ||E|| <= c eps sigma_0, so the subspaces are c eps sigma_0 /
    (sigma_{me-1} - sigma_me) apart (Wedin); applied to X the rotation mixes
    modes of size sigma_{me-1} at most, hence c eps sigma_{me-1} / gap
    relative to sigma_0 <= ||X||."""
    s = np.asarray(sigma, float)
    nxt = s[me] if me < s.size else 0.0
    gap = s[me - 1] - nxt
    return max(1e-12, c * 2.2e-16 * s[me - 1] / gap)


def validate_filter(prob, gamma, q_prev, passes_gpu, hp=None, tie_rel=1e-12):
    """Check a GPU filter run pass by pass against the oracle's gate on the
    same input.  ``gamma`` is the oracle's state before the filter (equal to
    the GPU's to rounding), ``passes_gpu`` the GPU's applied passes [(n,
    kept-cell mask)].  For every pass, on the state left by the previous
    passes (with the GPU's masks): the GPU's mask must equal the strict gate
    rf < r except at ties |rf - r| <= tie_rel max(1, |gamma|_inf) (where both
    flags are correct), and the loop control (orders, stop on an empty set,
    on a relative l1 decrease below eps_f, after j_max^f passes) must produce
    exactly the GPU's sequence of passes.  Returns (state after the GPU's
    passes, number of tied flags)."""
    from oracle import fv, hybrid
    hp = hp or hybrid.HybridParams()
    c = prob.ncomp
    g = gamma.copy()
    scale = max(1.0, float(np.max(np.abs(gamma))))
    k = 0
    ties = 0
    for n in hp.filter_orders:
        r = fv.cell_residual_norm(prob, g, q_prev)
        for it in range(1, hp.jfmax + 1):
            gf = hybrid.shapiro(prob, g, n)
            rf = fv.cell_residual_norm(prob, gf, q_prev)
            want = rf < r
            applied = k < len(passes_gpu) and passes_gpu[k][0] == n
            mk = np.asarray(passes_gpu[k][1], dtype=bool) if applied else np.zeros_like(want)
            flip = np.flatnonzero(mk != want)
            if flip.size:
                gap = np.abs(rf[flip] - r[flip])
                assert np.all(gap <= tie_rel * scale), ("gate", n, it, flip[gap > tie_rel * scale], gap.max())
                ties += int(flip.size)
            if applied:
                k += 1
            if not mk.any():
                break                       # an empty gate ends the order
            g = np.where(np.tile(mk, c), gf, g)
            r_new = fv.cell_residual_norm(prob, g, q_prev)
            s_old, s_new = np.sum(r), np.sum(r_new)
            r = r_new
            if (s_old - s_new) / s_old < hp.eps_f:
                break
    assert k == len(passes_gpu), ("pass count", k, len(passes_gpu))
    return g, ties
