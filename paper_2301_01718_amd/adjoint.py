"""Adjoint of the hybrid-snapshot trajectory with frozen decisions.

The trajectory map gamma_0 -> gamma_T of Alg. 1 contains decisions that have
no derivative: the step schedule, the sampled sets, the subiteration counts,
the filter masks and the bases (Phi_k, psi_k, which depend on earlier
snapshots).  The gradient computed here is that of the map with all of them
frozen at their forward values; every step is then a smooth function of its
input (eq. hdm for full steps; eq. hybrid with the subiterations of
Sec. 2.3.2 and the gated filters of Sec. 2.3.4 for hybrid steps).

The library does both directions: ``hs_traj_forward`` runs Alg. 1 and
records the frozen decisions and a checkpoint every K steps in a trajectory
tape; ``hs_traj_backward`` replays each segment from its checkpoint (checked
bit for bit against the next checkpoint) and applies the step adjoints in
reverse.  This module only marshals arguments and exposes the recorded run
for inspection.  ``HybridTrajectory.apply(q0, trajectory)`` exposes it to
torch.autograd.
"""
from __future__ import annotations

import time

import torch

from ._lib import (FP64, TAPE_REPLAY, Context, SampleParams, TrajParams, TrajTape, _ptr, hybrid_params, lib)
from .driver import AromConfig


def traj_params(cfg: AromConfig, steps: int, K: int, psi_adjoint: bool = False) -> TrajParams:
    tp = TrajParams()
    tp.steps, tp.checkpoint_every, tp.w, tp.m, tp.z = steps, K, cfg.w, cfg.m, cfg.z
    tp.psi_adjoint = 1 if psi_adjoint else 0
    tp.tau_pod = cfg.tau_pod
    tp.sample = SampleParams(rule=cfg.rule, fraction=cfg.fraction, delta=cfg.delta, halo=cfg.halo)
    tp.hybrid = hybrid_params(cfg.eps_y, cfg.jmax, cfg.filter_orders, cfg.eps_f, cfg.jfmax, cfg.rcond_fit,
                              cfg.floor_rel, FP64)
    return tp


class _Tapes:
    """tapes[k]: the recorded hybrid-step tape of step k (borrowed)."""

    def __init__(self, traj):
        self.traj = traj

    @property
    def tapes(self):
        return self.traj.tapes


class Trajectory:
    """An Alg.-1 trajectory of ``steps`` steps that can be differentiated.

    ``forward(q0)`` runs it (hs_traj_forward) and records the frozen
    decisions; ``backward(lam)`` returns (d gamma_T / d gamma_0)^T lam for
    the last forward run (hs_traj_backward; with ``psi_adjoint`` also through
    each hybrid step's reference state, the mean of the snapshots its basis
    update averaged, only the bases frozen).  After a forward run, ``kinds``
    (step -> ("full"|"hybrid", basis index)), ``bases`` (index -> (Phi,
    psi, m), copied on first use), ``tapes`` (step -> hybrid-step tape) and
    ``ckpt`` (checkpoint step -> state) expose the recorded run."""

    def __init__(self, prob, cfg: AromConfig, steps: int, checkpoint_every: int = 10, device="cuda",
                 ctx=None, psi_adjoint: bool = False):
        if checkpoint_every < 1:
            raise ValueError("checkpoint_every must be >= 1")
        if cfg.precision != FP64:
            raise ValueError("the adjoint runs on an FP64 basis (AromConfig.precision = FP64)")
        self.prob = prob
        self.cfg = cfg
        self.steps = steps
        self.K = checkpoint_every
        self.ctx = ctx or Context(prob, m_max=cfg.m, w_max=cfg.w, device=device)
        self.params = traj_params(cfg, steps, checkpoint_every, psi_adjoint)
        self.hp = self.params.hybrid
        self.tape = TrajTape(self.ctx)
        self.recorder = _Tapes(self)
        self.timing = {}
        self._reset()

    def _reset(self):
        self.kinds, self.tapes, self._bases, self._ckpt = {}, {}, {}, {}

    # ------------------------------------------------------------ forward
    def forward(self, q0):
        c = self.ctx
        q0 = c._in(q0.detach().contiguous())
        qT = c.empty()
        self._reset()
        torch.cuda.synchronize(c.device)
        t0 = time.perf_counter()
        c._check(lib().hs_traj_forward(c.h, _ptr(q0), self.params, self.tape.h, _ptr(qT)))
        self.timing["forward_s"] = time.perf_counter() - t0
        for k in range(1, self.steps + 1):
            kind, v, tape = self.tape.step(k)
            self.kinds[k] = ("hybrid", v) if kind == 1 else ("full", None)
            if tape is not None:
                self.tapes[k] = tape
        return qT

    # ----------------------------------------------------------- backward
    def backward(self, lam):
        c = self.ctx
        lam = c._in(lam.detach().to(torch.float64).contiguous())
        out = c.empty()
        torch.cuda.synchronize(c.device)
        t0 = time.perf_counter()
        c._check(lib().hs_traj_backward(c.h, self.tape.h, _ptr(lam), _ptr(out)))
        self.timing["backward_s"] = time.perf_counter() - t0
        return out

    # ------------------------------------------------------- inspection
    @property
    def bases(self):
        return _Lazy(self._bases, lambda v: self.tape.basis(v, self.cfg.m))

    @property
    def ckpt(self):
        return _Lazy(self._ckpt, self.tape.checkpoint)

    def _replay(self, s0, s1):
        """The states of steps s0+1..s1 replayed from checkpoint s0 with the
        recorded decisions through the step calls (inspection; the library's
        backward does the same internally); checked against checkpoint s1."""
        c = self.ctx
        q = self.ckpt[s0]
        outs = {}
        for k in range(s0 + 1, s1 + 1):
            kind, v = self.kinds[k]
            if kind == "full":
                out, _ = c.hdm_step(q)
            else:
                Phi, psi, m = self.bases[v]
                out, _ = c.rom_hybrid_step_taped(q, Phi, psi, m, self.tapes[k], TAPE_REPLAY, params=self.hp)
            outs[k] = out
            q = out
        if not torch.equal(q, self.ckpt[s1]):
            raise RuntimeError(f"replay of steps {s0 + 1}..{s1} did not reproduce the recorded state")
        return outs

    def decisions(self):
        """Per step: ("full", None) or ("hybrid", (tape, Phi, psi, m))."""
        out = []
        for k in range(1, self.steps + 1):
            kind, v = self.kinds[k]
            out.append((kind, None if kind == "full" else (self.tapes[k],) + self.bases[v]))
        return out


class _Lazy(dict):
    """A read-only mapping filled on first access of a key."""

    def __init__(self, cache, make):
        super().__init__()
        self._cache, self._make = cache, make

    def __getitem__(self, key):
        if key not in self._cache:
            self._cache[key] = self._make(key)
        return self._cache[key]


class HybridTrajectory(torch.autograd.Function):
    """gamma_T = HybridTrajectory.apply(gamma_0, trajectory); backward gives the
    frozen-decision gradient with respect to gamma_0."""

    @staticmethod
    def forward(fctx, q0, traj: Trajectory):
        fctx.traj = traj
        return traj.forward(q0)

    @staticmethod
    def backward(fctx, g):
        return fctx.traj.backward(g), None
