"""Host logic of the Algorithm-1 driver, without a GPU: a stand-in for the
library context records the calls, so the schedule, the update sequence and
the fallback of a failed hybrid step to a full step can be checked on the
CPU (the driver only sequences calls; the arithmetic is the library's)."""
import pytest
import torch

import paper_2301_01718_amd.driver as D
from paper_2301_01718_amd._lib import HsError, HS_ERR_NOT_CONVERGED, HS_ERR_RANK
from oracle import arom


class FakeSamples:
    def __init__(self):
        self.n_s = 5

    def counts(self):
        return {"n_g": 3, "n_s": self.n_s, "l": 2}


class FakeCtx:
    """Implements the Context methods the driver calls; a hybrid step raises
    ``fail`` on the steps listed in ``fail_at``."""

    def __init__(self, n, fail_at=(), fail=HS_ERR_NOT_CONVERGED):
        self.n = self.ncell = n
        self.device = torch.device("cpu")
        self.calls = []
        self.fail_at, self.fail = set(fail_at), fail
        self.k = 0
        self._pending = False

    def empty(self, n=None, dtype=torch.float64):
        return torch.zeros(self.n if n is None else n, dtype=dtype)

    def samples(self):
        return FakeSamples()

    def hdm_step(self, q_prev, out=None):
        self.calls.append("hdm_step")
        out.copy_(q_prev + 1.0)
        return out, {"newton_iters": 2, "lin_sweeps": 10}

    def rom_hybrid_step(self, q_prev, Phi, psi, m, samples, params=None, out=None, eps=None, y=None):
        self.calls.append("rom_hybrid_step")
        if m == D.BASIS_PENDING:
            self._pending = False
        if self.k in self.fail_at:
            raise HsError(self.fail, "forced")
        out.copy_(q_prev + 0.5)
        return out, {"n_s": 5, "l": 2, "subiters": 3, "newton_iters": 4, "lin_sweeps": 40, "filter_passes": 2,
                     "fit_cond": 1.0}

    def indicator_full(self, gamma, Phi, psi, m, floor_rel, eps=None):
        self.calls.append("indicator_full")

    def snapshot_table(self, window):
        return list(window)

    def basis_update_async(self, table, w, m, Phi, psi, sigma, tau):
        self.calls.append("basis_update")
        self._pending = True

    def basis_pending(self):
        return self._pending

    def basis_update_finish(self):
        self._pending = False
        return 3

    def basis_m_eff(self):
        return 3

    def sample_select(self, eps, fraction, halo, samples=None, rule=0, delta=0.9):
        self.calls.append("sample_select")


def run(steps, w, z, **kw):
    ctx = FakeCtx(8, **kw)
    drv = D.Arom(None, D.AromConfig(w=w, m=2, z=z), ctx=ctx)
    drv.start(torch.zeros(8, dtype=torch.float64), steps)
    recs = []
    for _ in range(steps):
        ctx.k = drv.k + 1
        recs.append(drv.advance())
    drv.finish()
    return ctx, recs


def test_schedule_matches_oracle_closed_form():
    w, z, steps = 6, 5, 23
    ctx, recs = run(steps, w, z)
    # hybrid wherever Alg. 1 allows one and a basis and sampled set exist
    for r in recs:
        k = r["k"]
        first_hybrid = w + 1            # the update after step w is the first with sampled sets
        want = "full" if (arom.is_full_step(k, w, z) or k < first_hybrid) else "hybrid"
        assert r["type"] == want, (k, r["type"])
    assert ctx.calls.count("basis_update") == sum(arom.wants_update(k, w, z, steps) for k in range(1, steps + 1))


@pytest.mark.parametrize("err", [HS_ERR_NOT_CONVERGED, HS_ERR_RANK])
def test_failed_hybrid_step_falls_back_to_a_full_step(err):
    w, z, steps = 6, 50, 14
    ctx, recs = run(steps, w, z, fail_at={9, 11}, fail=err)
    r9 = recs[8]
    assert r9["type"] == "full" and "fallback" in r9 and "forced" in r9["fallback"]
    assert recs[9]["type"] == "hybrid"          # the run goes on with hybrid steps
    assert recs[10]["type"] == "full" and "fallback" in recs[10]
    # the failed step was redone by a full solve on the same input
    i = [j for j, c in enumerate(ctx.calls) if c == "rom_hybrid_step"]
    assert ctx.calls[i[2] + 1] == "hdm_step"


def test_other_errors_propagate():
    w, z, steps = 6, 50, 10
    with pytest.raises(HsError):
        run(steps, w, z, fail_at={8}, fail=-6)


@pytest.mark.parametrize("kw", [dict(odeim_factor=2, m=17), dict(odeim_factor=2, m=4, precision=D.MIXED_FP32),
                                dict(gauss_newton=True, m=4, precision=D.MIXED_FP32)])
def test_unsupported_option_combinations_fail_before_any_allocation(kw):
    """ODEIM points need an FP64 basis of at most 16 modes and Gauss-Newton
    subiterations an FP64 basis: the driver says so at construction, before
    it creates a context or allocates device memory."""
    with pytest.raises(ValueError):
        D.Arom(None, D.AromConfig(w=6, z=5, **kw), ctx=None)


def test_gauss_newton_with_the_paper_scheme_fails_at_construction():
    with pytest.raises(ValueError):
        D.Arom(None, D.AromConfig(w=6, m=4, z=5, gauss_newton=True), ctx=None, paper=object())
