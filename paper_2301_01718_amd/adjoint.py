"""Adjoint of the hybrid-snapshot trajectory with frozen decisions.

The trajectory map gamma_0 -> gamma_T of Alg. 1 contains decisions that have
no derivative: the step schedule, the sampled sets, the subiteration counts,
the filter masks and the bases (Phi_k, psi_k, which depend on earlier
snapshots).  The gradient computed here is that of the map with all of them
frozen at their forward values; every step is then a smooth function of its
input (eq. hdm for full steps; eq. hybrid with the subiterations of
Sec. 2.3.2 and the gated filters of Sec. 2.3.4 for hybrid steps).

Forward: the driver runs Alg. 1; each hybrid step records its decisions in a
library tape and the basis it used is kept; the state is checkpointed every K
steps.  Backward: per segment of K steps, last first, the segment is
replayed from its checkpoint (full steps re-solved, hybrid steps in tape
replay mode, which reproduces the recorded outputs bit for bit and keeps each
subiteration's state), then the step adjoints run in reverse order through
``hdm_step_adjoint`` and ``rom_hybrid_step_adjoint``.

``HybridTrajectory.apply(q0, trajectory)`` exposes it to torch.autograd.
"""
from __future__ import annotations

import time

import torch

from ._lib import FP64, TAPE_REPLAY
from .driver import Arom, AromConfig


class _Recorder:
    """Hands the driver one library tape per hybrid step (reused across runs)."""

    def __init__(self, ctx):
        self.ctx = ctx
        self.tapes = {}

    def tape(self, k):
        t = self.tapes.get(k)
        if t is None:
            t = self.ctx.tape()
            self.tapes[k] = t
        return t


class Trajectory:
    """An Alg.-1 trajectory of ``steps`` steps that can be differentiated.

    ``forward(q0)`` runs it and records the frozen decisions; ``backward(lam)``
    returns (d gamma_T / d gamma_0)^T lam for the last forward run."""

    def __init__(self, prob, cfg: AromConfig, steps: int, checkpoint_every: int = 10, device="cuda",
                 ctx=None, verify_replay: bool = True):
        if checkpoint_every < 1:
            raise ValueError("checkpoint_every must be >= 1")
        if cfg.precision != FP64:
            raise ValueError("the adjoint runs on an FP64 basis (AromConfig.precision = FP64)")
        self.prob = prob
        self.cfg = cfg
        self.steps = steps
        self.K = checkpoint_every
        self.drv = Arom(prob, cfg, device=device, ctx=ctx)
        self.ctx = self.drv.ctx
        self.recorder = _Recorder(self.ctx)
        self.verify_replay = verify_replay
        self.records = []
        self.timing = {}

    # ------------------------------------------------------------ forward
    def forward(self, q0):
        c = self.ctx
        q0 = c._in(q0.detach().contiguous())
        self.ckpt = {0: q0.clone()}
        self.kinds = {}
        self.bases = {}
        K = self.K

        def on_step(k, rec, used, out):
            if rec["type"] == "hybrid":
                v = used["basis_version"]
                if v not in self.bases:
                    m = used["m"]
                    self.bases[v] = (used["Phi"][: m * c.n].clone(), used["psi"].clone(), m)
                self.kinds[k] = ("hybrid", v)
            else:
                self.kinds[k] = ("full", None)
            if k % K == 0 or k == self.steps:
                self.ckpt[k] = out.clone()

        self.drv.recorder = self.recorder
        torch.cuda.synchronize(c.device)
        t0 = time.perf_counter()
        try:
            qT, self.records = self.drv.run(q0, self.steps, on_step=on_step)
        finally:
            self.drv.recorder = None
        torch.cuda.synchronize(c.device)
        self.timing["forward_s"] = time.perf_counter() - t0
        return self.ckpt[self.steps].clone()

    # ----------------------------------------------------------- backward
    def _replay(self, s0, s1):
        c = self.ctx
        q = self.ckpt[s0]
        outs = {}
        for k in range(s0 + 1, s1 + 1):
            kind, v = self.kinds[k]
            if kind == "full":
                out, _ = c.hdm_step(q)
            else:
                Phi, psi, m = self.bases[v]
                out, _ = c.rom_hybrid_step_taped(q, Phi, psi, m, self.recorder.tapes[k], TAPE_REPLAY,
                                                 params=self.drv.hp)
            outs[k] = out
            q = out
        if self.verify_replay and not torch.equal(q, self.ckpt[s1]):
            raise RuntimeError(f"replay of steps {s0 + 1}..{s1} did not reproduce the recorded state")
        return outs

    def backward(self, lam):
        c = self.ctx
        lam = c._in(lam.detach().to(torch.float64).contiguous()).clone()
        torch.cuda.synchronize(c.device)
        t0 = time.perf_counter()
        sweeps = 0
        for s0 in reversed(range(0, self.steps, self.K)):
            s1 = min(s0 + self.K, self.steps)
            outs = self._replay(s0, s1)
            for k in range(s1, s0, -1):
                kind, v = self.kinds[k]
                if kind == "full":
                    lam, info = c.hdm_step_adjoint(outs[k], lam)
                else:
                    Phi, _, m = self.bases[v]
                    lam, info = c.rom_hybrid_step_adjoint(Phi, m, self.recorder.tapes[k], lam)
                sweeps += info["lin_sweeps"]
            del outs
        torch.cuda.synchronize(c.device)
        self.timing["backward_s"] = time.perf_counter() - t0
        self.timing["adjoint_sweeps"] = sweeps
        return lam

    def decisions(self):
        """Per step: ("full", None) or ("hybrid", (tape, Phi, psi, m))."""
        out = []
        for k in range(1, self.steps + 1):
            kind, v = self.kinds[k]
            out.append((kind, None if kind == "full" else (self.recorder.tapes[k],) + self.bases[v]))
        return out


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
