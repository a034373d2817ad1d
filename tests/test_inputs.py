"""The seeded generators are reproducible: digests stored by
tests/golden/make_input_digests.py must be regenerated bit for bit."""
import json
import os

import numpy as np
import pytest

import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "input_digests.json")))


@pytest.mark.parametrize("key", sorted(k for k in GOLD if not k.startswith("burgers1d_256k")
                                        and not k.startswith("burgers2d_1024") and "/" in k
                                        and not k.startswith(("paper/", "random_euler/"))) + ["burgers2d_1024/0"])
def test_input_digest(key):
    name, seed = key.split("/")
    prob, q0 = W.make(W.WORKLOADS[name], int(seed))
    assert W.digest(q0) == GOLD[key]["sha256"]
    assert prob.dt == GOLD[key]["dt"]


def test_workload_shapes():
    wl = W.WORKLOADS["burgers2d_1024"]
    assert (wl.ncell, wl.m, wl.w, wl.z) == (1 << 20, 32, 48, 20)
    assert W.WORKLOADS["euler2d_512"].n == 4 * 512 * 512
    assert W.WORKLOADS["burgers1d_1k"].w == 15


def test_euler_states_in_ranges():
    rng = np.random.default_rng(0)
    for rho, p, u, v in W.euler_quadrant_states(rng):
        assert 0.1 <= rho <= 1.5 and 0.03 <= p <= 1.5 and abs(u) <= 1.2 and abs(v) <= 1.2


@pytest.mark.parametrize("name", ["sod", "implosion"])
def test_paper_case_digest(name):
    case = W.paper_sod() if name == "sod" else W.paper_implosion()
    g = GOLD[f"paper/{name}"]
    assert W.digest(case.q0) == g["sha256"]
    assert (case.dt, case.nx, case.ny) == (g["dt"], g["nx"], g["ny"])


@pytest.mark.parametrize("key", sorted(k for k in GOLD if k.startswith("random_euler/")))
def test_random_euler_state_digest(key):
    _, shape, seed = key.split("/")
    nx, ny = (int(t) for t in shape.split("x"))
    assert W.digest(W.random_euler_state(nx, ny, int(seed))) == GOLD[key]["sha256"]
