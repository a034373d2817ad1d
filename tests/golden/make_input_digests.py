"""Writes input_digests.json: SHA-256 of every workload's initial state for
seeds 0-4.  Calls only the input generators (no method arithmetic)."""
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
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "input_digests.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
