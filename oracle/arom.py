"""Algorithm 1 (hybrid snapshot AROM) and the run statistics (oracle; test use only).

Paper passages followed
-----------------------
* Algorithm 1: full HDM solves for the first w-1 steps and every z steps,
  hybrid steps otherwise; the reference state at k = w-1; sampling, basis
  and reference-state updates after step k when k >= w-1 and step k+1 is
  not a full step; G empty at k = w-1 (Sec. 2.4.1).
* Error and sampling statistics: e_k, e-bar, s-bar, s-bar* (Sec. 3.1).

Readings
--------
* A step whose sampled set is empty (or that has no basis) is a full step;
  this covers k = w, since without ODEIM points the sampled set built at
  k = w-1 is empty.
* After a full step the indicator uses the latest basis and reference state
  with y = Phi^T (gamma - psi); the centring state of a basis update is the
  mean of the w snapshots before the newest (computed from the window, which
  equals the stored reference state whenever Alg. 1 stored one).
* The update after the last step is not needed and is skipped.
* A hybrid step whose Newton solve fails falls back to a full step.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from workloads import Problem

from . import fv, pod, sampling
from .hybrid import HybridParams, hybrid_step


@dataclasses.dataclass
class AromParams:
    w: int
    m: int
    z: int = 20
    rule: int = sampling.RULE_FRACTION
    fraction: float = 0.1
    delta: float = 0.9
    halo: int = 2
    tau_pod: float = pod.DEFAULT_TAU
    hybrid: HybridParams = dataclasses.field(default_factory=HybridParams)


def is_full_step(k, w, z):
    """The schedule part of Alg. 1's full/hybrid test."""
    return k + 1 <= w or k % z == 0


def wants_update(k, w, z, steps):
    return k >= w - 1 and (k + 1) % z != 0 and k < steps


def run(prob: Problem, q0, steps, p: AromParams, keep_all=False, on_step=None):
    """Run Alg. 1 for ``steps`` steps.  Returns a dict with the final state,
    per-step records and (if keep_all) every snapshot."""
    gammas = [q0.copy()]
    basis = None            # (Phi, psi) latest
    samples = None          # sampled sets for the next step
    records = []
    for k in range(1, steps + 1):
        rec = {"k": k}
        hybrid_ok = (not is_full_step(k, p.w, p.z) and samples is not None
                     and samples["hat"].size > 0 and basis is not None
                     and basis[0].shape[1] > 0)
        eps = None
        if hybrid_ok:
            try:
                out = hybrid_step(prob, gammas[-1], basis[0], basis[1],
                                  samples["hat"], samples["tilde"], p.hybrid)
                g = out["gamma"]
                eps = out["eps"]
                rec.update(type="hybrid", n_s=int(samples["hat"].size),
                           l=int(samples["tilde"].size), J=out["J"],
                           newton=out["newton"])
            except fv.NotConverged:
                hybrid_ok = False
        if not hybrid_ok:
            g, its = fv.hdm_step(prob, gammas[-1])
            rec.update(type="full", n_s=prob.ncell, newton=[its])
        gammas.append(g)
        if not keep_all and len(gammas) > p.w + 2:
            gammas[-(p.w + 3)] = None
        samples = None
        if wants_update(k, p.w, p.z, steps):
            if k >= p.w and basis is not None and basis[0].shape[1] > 0:
                if eps is None:
                    eps, _ = sampling.indicator_full(prob, g, basis[0], basis[1],
                                                     p.hybrid.floor_rel)
                samples = sampling.select(prob, eps, p.rule, p.fraction, p.delta, p.halo)
                rec["n_g"] = samples["n_g"]
            window = gammas[k - p.w:k + 1] if k >= p.w else gammas[0:k + 1]
            b = pod.pod(window, p.w, p.m, p.tau_pod)
            basis = (b["Phi"], b["psi_new"])
            rec["m_eff"] = b["m_eff"]
        records.append(rec)
        if on_step is not None:
            on_step(k, g, rec)
    return {"q": gammas[-1], "records": records,
            "gammas": gammas if keep_all else None}


def relative_l1_error(gamma, q):
    """e_k: relative L1 error of a snapshot against the full-HDM state (uniform cells)."""
    return float(np.sum(np.abs(gamma - q)) / np.sum(np.abs(q)))


def sampling_stats(prob: Problem, records):
    """s-bar (all steps) and s-bar* (hybrid steps) as fractions of N."""
    n = prob.ncell
    frac = [r["n_s"] / n for r in records]
    hyb = [r["n_s"] / n for r in records if r["type"] == "hybrid"]
    return float(np.mean(frac)), (float(np.mean(hyb)) if hyb else float("nan"))
