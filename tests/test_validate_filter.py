"""The pass-by-pass filter checker of the GPU tests (gpu_common.validate_filter),
on the CPU: it accepts the oracle's own passes (zero ties, the same state to
the bit) and rejects a flag flipped where the gate is not a tie, a pass of
the wrong order and a missing pass."""
import numpy as np
import pytest

import workloads as W
from oracle import fv, hybrid, pod, sampling

from gpu_common import validate_filter


@pytest.fixture(scope="module")
def filtered():
    wl = W.WORKLOADS["euler2d_512"].resized(40, 36)
    prob, q0 = W.make(wl, 0)
    snaps = [q0]
    for _ in range(12):
        snaps.append(fv.hdm_step(prob, snaps[-1])[0])
    b = pod.pod(snaps, 12, 8)
    eps, _ = sampling.indicator_full(prob, snaps[-1], b["Phi"], b["psi_new"])
    sel = sampling.select(prob, eps, 0, 0.08)
    args = (prob, snaps[-1], b["Phi"], b["psi_new"], sel["hat"], sel["tilde"])
    ref = hybrid.hybrid_step(*args)
    pre = hybrid.hybrid_step(*args, hybrid.HybridParams(filter_orders=()))["gamma"]
    assert len(ref["masks"]) >= 3
    return prob, snaps[-1], pre, ref


def test_accepts_the_oracles_own_passes(filtered):
    prob, q_prev, pre, ref = filtered
    g, ties = validate_filter(prob, pre, q_prev, ref["masks"])
    assert ties == 0 and np.array_equal(g, ref["gamma"])


def test_rejects_a_flag_that_is_not_a_tie(filtered):
    prob, q_prev, pre, ref = filtered
    masks = [(n, m.copy()) for n, m in ref["masks"]]
    n, m = masks[1]
    m[np.flatnonzero(m)[0]] = False
    with pytest.raises(AssertionError):
        validate_filter(prob, pre, q_prev, masks)


def test_rejects_a_wrong_order_or_a_missing_pass(filtered):
    prob, q_prev, pre, ref = filtered
    masks = [(n, m.copy()) for n, m in ref["masks"]]
    with pytest.raises(AssertionError):
        validate_filter(prob, pre, q_prev, [(masks[0][0] % 3 + 1, masks[0][1])] + masks[1:])
    with pytest.raises(AssertionError):
        validate_filter(prob, pre, q_prev, masks[:-1])
