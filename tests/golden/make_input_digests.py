"""Writes input_digests.json: SHA-256 of every workload's initial state for
seeds 0-4, of the paper's two experiments' initial states (Sod's tube,
Sec. 3.2; the model implosion, Sec. 3.3) at full size, and of the seeded
random Euler states of the paper-scheme parity tests.  Calls only the input
generators (no method arithmetic)."""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import workloads as W  # noqa: E402


def main():
    out = {}
    for name, wl in W.WORKLOADS.items():
        for seed in range(5):
            prob, q0 = W.make(wl, seed)
            out[f"{name}/{seed}"] = {"sha256": W.digest(q0), "dt": prob.dt, "inflow": prob.inflow}
    for case in (W.paper_sod(), W.paper_implosion()):
        out[f"paper/{case.name}"] = {"sha256": W.digest(case.q0), "dt": case.dt, "nx": case.nx, "ny": case.ny}
    for nx, ny in ((1237, 1), (45, 37)):
        for seed in range(3):
            out[f"random_euler/{nx}x{ny}/{seed}"] = {"sha256": W.digest(W.random_euler_state(nx, ny, seed))}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "input_digests.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
