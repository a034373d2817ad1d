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


def indicator_close(eg, eo, gamma, floor_rel=1e-11, tol=1e-13):
    """Compare two indicators cell by cell through the error norms sqrt(eps):
    eps is the square of a difference of nearly equal states, so its
    reproducible part is the norm, accurate to a few ulps of the state scale.
    A cell may flip between flushed and kept only within 1 % of the floor."""
    scale = max(1.0, float(np.max(np.abs(gamma))))
    fl = floor_rel * scale
    a, b = np.sqrt(eg), np.sqrt(eo)
    near_floor = (np.minimum(np.where(a > 0, a, np.inf), np.where(b > 0, b, np.inf)) < 1.01 * fl)
    bad = (np.abs(a - b) > tol * scale) & ~near_floor
    return not bad.any(), float(np.max(np.abs(a - b)) / scale)


def projector_tol(sigma, me, c=10.0):
    """Bound on ||P_gpu X - P_oracle X|| / ||X|| for two rank-me POD projectors
    built from the same window: both are within c * eps * lambda_0 of the exact
    Gram matrix, so the projector moves by at most that over the eigenvalue gap
    at the cut, (lambda_{me-1} - lambda_me) (Davis-Kahan)."""
    lam = np.asarray(sigma, float) ** 2
    nxt = lam[me] if me < lam.size else 0.0
    gap = (lam[me - 1] - nxt) / lam[0]
    return max(1e-12, c * 2.2e-16 / gap)
