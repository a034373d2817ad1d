"""Algorithm 1 (hybrid snapshot AROM) on the GPU library.

The driver only sequences the four calls of the C ABI (hdm_step,
sample_select, rom_hybrid_step, basis_update; with the paper's own scheme
hdm_step_bdf2 and rom_hybrid_step_bdf2, which also take gamma_{k-2}) and
keeps the window of the
last w + 1 snapshots resident in HBM as a ring of device buffers.  The
schedule follows Alg. 1: full solves for the first w - 1 steps and every z
steps; after step k (k >= w - 1, step k + 1 not full) the indicator of the
newest snapshot selects the sampled set of step k + 1 and the basis and
reference state are rebuilt from the window.  A step whose sampled set is
empty, or that has no basis, is a full step; a hybrid step whose Newton solve
fails is redone as a full step.
"""
from __future__ import annotations

import dataclasses
import time

import torch

from ._lib import (BASIS_PENDING, Context, HsError, FP64, HS_ERR_NOT_CONVERGED, HS_ERR_RANK, MIXED_FP32,
                   RULE_FRACTION, TAPE_RECORD, hybrid_params)


@dataclasses.dataclass
class AromConfig:
    w: int
    m: int
    z: int = 20
    fraction: float = 0.1
    halo: int = 2
    rule: int = RULE_FRACTION      # or RULE_RRE (eq. rre) with delta
    delta: float = 0.9
    tau_pod: float = 1e-8
    eps_y: float = 1e-4
    jmax: int = 10
    filter_orders: tuple = (1, 2, 3)
    eps_f: float = 1e-2
    jfmax: int = 10
    rcond_fit: float = 1e-8
    floor_rel: float = 1e-14
    precision: int = FP64
    # ODEIM points (eq. odeim), n_p = odeim_factor m_eff, join the sampled set
    # and are the fit's rows (eq. red_coord); 0: none (FP64 basis)
    odeim_factor: int = 0
    # Gauss-Newton subiterations (rom_hybrid_step_gn; first-order scheme, FP64)
    gauss_newton: bool = False


def is_full_step(k, w, z):
    return k + 1 <= w or k % z == 0


def wants_update(k, w, z, steps):
    return k >= w - 1 and (k + 1) % z != 0 and k < steps


ODEIM_MAX_MODES = 16   # the largest basis hs_odeim takes


class Arom:
    """Runs Alg. 1 on one device.  ``on_step(k, rec, used, out)`` is called
    after every step with the step record, the device tensors the step used
    and its output; ``on_update(k, rec, state)`` after every sampling/basis
    update.  The tensors are valid only during the call."""

    RING_STAGGER = 320   # doubles between consecutive ring slots beyond N (2560 B: whole 128-B lines)

    def __init__(self, prob, cfg: AromConfig, device="cuda", ctx: Context | None = None, paper=None):
        if cfg.odeim_factor > 0 and (cfg.precision != FP64 or cfg.m > ODEIM_MAX_MODES):
            raise ValueError(f"ODEIM points need an FP64 basis of at most {ODEIM_MAX_MODES} modes")
        if cfg.gauss_newton and (cfg.precision != FP64 or paper is not None):
            raise ValueError("Gauss-Newton subiterations run with the first-order scheme on an FP64 basis")
        self.prob = prob
        self.cfg = cfg
        self.ctx = ctx or Context(prob, m_max=cfg.m, w_max=cfg.w, device=device)
        c = self.ctx
        # the snapshot ring: one allocation, slots staggered by a few KiB so
        # that the same row of different snapshots does not map to the same
        # HBM channel (the basis passes read one row of every slot at once)
        nslot = cfg.w + 2
        stride = c.n + self.RING_STAGGER
        self._ring_buf = torch.empty(nslot * stride, dtype=torch.float64, device=c.device)
        self.ring = [self._ring_buf[j * stride: j * stride + c.n] for j in range(nslot)]
        self._tables = {}   # (first slot, length) -> the window's snapshot table
        # the basis: FP64, or its FP32 master copy in the mixed mode
        phi_dtype = torch.float32 if cfg.precision == MIXED_FP32 else torch.float64
        self.Phi = torch.zeros(cfg.m * c.n, dtype=phi_dtype, device=c.device)
        self.psi = c.empty()
        self.sigma = torch.zeros(cfg.w, dtype=torch.float64, device=c.device)
        self.eps = c.empty(c.ncell)
        self.samples = c.samples()
        self.hp = hybrid_params(cfg.eps_y, cfg.jmax, cfg.filter_orders, cfg.eps_f, cfg.jfmax,
                                cfg.rcond_fit, cfg.floor_rel, cfg.precision)
        self.m_eff = 0
        self.basis_version = 0
        # a basis update left in flight for the next hybrid step to complete
        # (after its first Newton solve, which does not need the basis)
        self.pending = None
        self.defer_basis = True
        # optional: an object with tape(k) -> Tape, called for every hybrid
        # step; the step then records its frozen decisions (adjoint use)
        self.recorder = None
        # the paper's own scheme (a PaperHDM: MUSCL + minmod, Roe, BDF2 with
        # gamma_{k-2}, Sec. 3.1) instead of the first-order one; its steps
        # take the basis once the update is complete
        self.paper = paper
        if paper is not None or cfg.odeim_factor > 0:
            self.defer_basis = False   # these steps take the basis (and its points) complete
        self.points = None
        self.gn_work = None
        if cfg.gauss_newton:
            self.gn_work = c.empty(cfg.m * c.n)
            self.defer_basis = False

    def slot(self, k):
        return self.ring[k % (self.cfg.w + 2)]

    def _complete(self):
        """Finish a pending basis update (if any) and record its m_eff."""
        if self.pending is not None:
            rec, self.pending = self.pending, None
            self.m_eff = self.ctx.basis_update_finish() if self.ctx.basis_pending() else self.ctx.basis_m_eff()
            rec["m_eff"] = self.m_eff

    def start(self, q0, steps):
        """Load gamma_0 and reset the schedule for a run of ``steps`` steps."""
        self._complete()
        self.slot(0).copy_(q0)
        self.m_eff = 0
        self.have_samples = False
        self.k = 0
        self.steps = steps

    def advance(self, on_step=None, on_update=None):
        """Compute step k+1 of Alg. 1 and the updates that follow it."""
        cfg, c = self.cfg, self.ctx
        self.k += 1
        k = self.k
        rec = {"k": k}
        prev, out = self.slot(k - 1), self.slot(k)
        hybrid = (not is_full_step(k, cfg.w, cfg.z) and self.have_samples
                  and (self.pending is not None or self.m_eff > 0))
        if not hybrid:
            self._complete()
        used = {"q_prev": prev, "Phi": self.Phi, "psi": self.psi, "m": self.m_eff,
                "basis_version": self.basis_version}
        prev2 = self.slot(k - 2) if k >= 2 else None
        if hybrid:
            m_arg = BASIS_PENDING if self.pending is not None else self.m_eff
            try:
                if self.paper is not None:
                    _, info = c.rom_hybrid_step_bdf2(self.paper, prev, prev2, self.Phi, self.psi, self.m_eff,
                                                     self.samples, self.hp, out=out, eps=self.eps,
                                                     fit_points=self.points)
                    rec["n_p"] = 0 if self.points is None else self.points.numel()
                elif self.gn_work is not None:
                    _, info = c.rom_hybrid_step_gn(prev, self.Phi, self.psi, self.m_eff, self.samples, self.hp,
                                                   out=out, eps=self.eps, work=self.gn_work)
                elif self.recorder is not None:
                    if self.points is not None:
                        raise ValueError("a taped hybrid step fits over the sampled cells (no ODEIM points)")
                    _, info = c.rom_hybrid_step_taped(prev, self.Phi, self.psi, m_arg,
                                                      self.recorder.tape(k), TAPE_RECORD,
                                                      samples=self.samples, params=self.hp, out=out,
                                                      eps=self.eps)
                else:
                    fit = {} if self.points is None else {"fit_points": self.points}
                    _, info = c.rom_hybrid_step(prev, self.Phi, self.psi, m_arg, self.samples,
                                                self.hp, out=out, eps=self.eps, **fit)
                rec.update(type="hybrid", n_s=info["n_s"], l=info["l"], J=info["subiters"],
                           newton=info["newton_iters"], sweeps=info["lin_sweeps"],
                           filter_passes=info["filter_passes"], fit_cond=info["fit_cond"])
            except HsError as e:
                if e.status not in (HS_ERR_NOT_CONVERGED, HS_ERR_RANK):
                    raise
                hybrid = False
                rec["fallback"] = str(e)
            finally:
                self._complete()        # the step completed the update on every path
                used["m"] = self.m_eff
        if not hybrid and self.paper is not None:
            _, info = c.hdm_step_bdf2(self.paper, prev, prev2, out=out)
            rec.update(type="full", n_s=c.ncell, newton=info["newton_iters"], sweeps=info["lin_sweeps"])
        elif not hybrid:
            _, info = c.hdm_step(prev, out=out)
            rec.update(type="full", n_s=c.ncell, newton=info["newton_iters"], sweeps=info["lin_sweeps"])
        if on_step is not None:
            used["samples"] = self.samples if hybrid else None
            on_step(k, rec, used, out)
        self.have_samples = False
        if wants_update(k, cfg.w, cfg.z, self.steps):
            sample = k >= cfg.w and self.m_eff > 0
            if sample and not hybrid:
                # the indicator of a full snapshot reads the current basis: before it is replaced
                c.indicator_full(out, self.Phi, self.psi, self.m_eff, cfg.floor_rel, eps=self.eps)
            lo = k - cfg.w if k >= cfg.w else 0
            window = [self.slot(j) for j in range(lo, k + 1)]
            # the basis update runs on the context's second stream while the
            # sampled sets are selected on its main stream
            key = (lo % (cfg.w + 2), len(window))
            table = self._tables.get(key)
            if table is None:
                table = self._tables[key] = c.snapshot_table(window)
            c.basis_update_async(table, cfg.w, cfg.m, self.Phi, self.psi, self.sigma, cfg.tau_pod)
            self.pending = rec
            try:
                if sample:
                    c.sample_select(self.eps, cfg.fraction, cfg.halo, samples=self.samples, rule=cfg.rule,
                                    delta=cfg.delta)
                    cnt = self.samples.counts()
                    rec["n_g"] = cnt["n_g"]
                    self.have_samples = cnt["n_s"] > 0
            finally:
                # left in flight only for a next step that is hybrid and can
                # complete it; a caller that inspects the update gets it whole
                nxt_hybrid = (not is_full_step(k + 1, cfg.w, cfg.z) and self.have_samples and k < self.steps)
                if on_update is not None or not self.defer_basis or not nxt_hybrid:
                    self._complete()
            self.points = None
            if cfg.odeim_factor > 0 and self.have_samples and self.m_eff > 0:
                # P_{k+1} = ODEIM(Phi_{k+1}) and hat-S = G u P (Alg. 1), the basis complete
                n_p = min(cfg.odeim_factor * self.m_eff, c.n)
                self.points = c.odeim(self.Phi, self.m_eff, n_p)
                c.samples_add_points(self.samples, self.points)
            self.basis_version += 1
            if on_update is not None:
                on_update(k, rec, {"eps": self.eps, "samples": self.samples if self.have_samples else None,
                                   "window": window, "Phi": self.Phi, "psi": self.psi,
                                   "sigma": self.sigma, "m_eff": self.m_eff, "points": self.points})
        return rec

    def state(self):
        return self.slot(self.k)

    def finish(self):
        """Complete a basis update still in flight (the end of a run)."""
        self._complete()

    def run(self, q0, steps, on_step=None, on_update=None, timing=False):
        self.start(q0, steps)
        records = []
        for _ in range(steps):
            t0 = time.perf_counter() if timing else 0.0
            rec = self.advance(on_step, on_update)
            if timing:
                torch.cuda.synchronize(self.ctx.device)
                rec["seconds"] = time.perf_counter() - t0
            records.append(rec)
        self._complete()
        return self.slot(steps), records
