"""The adjoint on 2D Burgers 256 x 256 over 100 steps, a
checkpoint every 10 steps, loss 0.5 ||u_T - u_target||^2 with u_target a
full-HDM run of 100 steps from the seed + 1 initial state.

* Central differences of the GPU's frozen trajectory map (every step
  replayed with the recorded decisions), h = 1e-6, 16 seeded directions:
  |g.d - FD| <= 1e-6 max(|g.d|, 1e-8 |g| |d|).
* Step by step against the oracle adjoint, resynchronised: walking the
  checkpointed segments backwards as the GPU does, every hybrid step's and
  every eighth full step's adjoint lambda_{k-1} is recomputed by the oracle
  from the GPU's lambda_k, the GPU's input gamma_{k-1} and the step's frozen
  decisions (sets, J, filter masks, basis), 1e-10 relative (C-12 (iii));
  the oracle's replay of each hybrid step from the same input equals the
  GPU's replayed output to 1e-12.
(The target, the states and the lambdas fed to the oracle are the GPU's, as
in the trajectory resynchronisation; each check is of one step's map.)"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as A
from oracle import hybrid

from gpu_common import dev, host, need_gpu, print_case, rel, torch

pytestmark = pytest.mark.gpu


def test_c4_gradient_full_size():
    need_gpu()
    print_case("adjoint: burgers2d 256^2, 100 steps, K = 10")
    from paper_2301_01718_amd._lib import TAPE_REPLAY
    from paper_2301_01718_amd.adjoint import HybridTrajectory, Trajectory
    from paper_2301_01718_amd.driver import AromConfig
    wl = W.WORKLOADS["burgers2d_256"]
    prob, q0 = W.make(wl, 0)
    _, q0t = W.make(wl, 1)
    cfg = AromConfig(w=wl.w, m=wl.m, z=wl.z, fraction=wl.frac, halo=wl.halo)
    traj = Trajectory(prob, cfg, wl.steps, checkpoint_every=wl.checkpoint)
    c = traj.ctx
    tgt = dev(q0t)
    for _ in range(wl.steps):
        tgt, _ = c.hdm_step(tgt)
    q = dev(q0).requires_grad_(True)
    qT = HybridTrajectory.apply(q, traj)
    loss = 0.5 * torch.sum((qT - tgt) ** 2)
    loss.backward()
    g = host(q.grad)
    kinds = [traj.kinds[k][0] for k in range(1, wl.steps + 1)]
    print(f"  steps {wl.steps}, hybrid {kinds.count('hybrid')}, |g| {np.linalg.norm(g):.6e}", flush=True)
    assert kinds.count("hybrid") > 20

    # central differences of the frozen GPU map
    def replay(q0p):
        x = dev(q0p)
        for k in range(1, wl.steps + 1):
            kind, v = traj.kinds[k]
            if kind == "full":
                x, _ = c.hdm_step(x)
            else:
                Phi, psi, m = traj.bases[v]
                x, _ = c.rom_hybrid_step_taped(x, Phi, psi, m, traj.recorder.tapes[k], TAPE_REPLAY,
                                               params=traj.hp)
        return x

    assert torch.equal(replay(q0), qT.detach())
    rng = np.random.default_rng(2)
    h = 1e-6
    worst = 0.0
    for i in range(16):
        d = rng.standard_normal(prob.n)
        # L(+) - L(-) = sum (u+ - u-) ((u+ + u-) / 2 - target): the same
        # difference without cancelling two loss values of size |L| (whose
        # own summation rounding, eps |L| / h, would exceed the bar)
        up, um = replay(q0 + h * d), replay(q0 - h * d)
        fd = float(torch.sum((up - um) * (0.5 * (up + um) - tgt))) / (2 * h)
        gd = float(g @ d)
        err = abs(gd - fd) / max(abs(gd), 1e-8 * np.linalg.norm(g) * np.linalg.norm(d))
        worst = max(worst, err)
        assert err <= 1e-6, (i, gd, fd)
    print(f"  16 directions: max relative FD difference {worst:.2e}", flush=True)

    # the adjoint step by step against the oracle, resynchronised
    hp = hybrid.HybridParams()
    lam = (qT.detach() - tgt).clone()
    checked = {"full": 0, "hybrid": 0}
    worst = {"full": 0.0, "hybrid": 0.0, "replay": 0.0}
    K = traj.K
    for s0 in reversed(range(0, wl.steps, K)):
        s1 = min(s0 + K, wl.steps)
        outs = traj._replay(s0, s1)
        outs[s0] = traj.ckpt[s0]
        for k in range(s1, s0, -1):
            kind, v = traj.kinds[k]
            lam_in = host(lam)
            if kind == "full":
                lam, _ = c.hdm_step_adjoint(outs[k], lam)
                if k % 8 == 0 or k == wl.steps:
                    ref = A.step_adjoint(prob, {"type": "full", "out": host(outs[k])}, lam_in, hp)
                    e = rel(host(lam), ref)
                    worst["full"] = max(worst["full"], e)
                    checked["full"] += 1
                    assert e <= 1e-10, (k, "full", e)
            else:
                Phi, psi, m = traj.bases[v]
                tape = traj.recorder.tapes[k]
                lam, _ = c.rom_hybrid_step_adjoint(Phi, m, tape, lam)
                hat, tilde, _ = (host(x) for x in tape.samples().export())
                J, passes = tape.info()
                st = {"type": "hybrid", "hat": hat, "tilde": tilde, "J": J,
                      "Phi": host(Phi).reshape(m, prob.n).T.copy(), "psi": host(psi),
                      "masks": [(n, host(mk).astype(bool)) for n, mk in passes]}
                out_o, st["us"] = A.replay_hybrid(prob, host(outs[k - 1]), st, hp, states=True)
                worst["replay"] = max(worst["replay"], rel(host(outs[k]), out_o))
                assert rel(host(outs[k]), out_o) <= 1e-12, (k, "replay")
                ref = A.step_adjoint(prob, st, lam_in, hp)
                e = rel(host(lam), ref)
                worst["hybrid"] = max(worst["hybrid"], e)
                checked["hybrid"] += 1
                assert e <= 1e-10, (k, "hybrid", e)
        print(f"  segment {s0 + 1}..{s1}: checked {checked}, worst {worst}", flush=True)
        del outs
    assert rel(host(lam), g) <= 1e-12          # the walk reproduces the autograd gradient
