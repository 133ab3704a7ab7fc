"""Write the stored expected values of tests/golden/ from the FP64 oracle.

Calls only castgen (inputs) and oracle/ (the CPU reference).  Run from the
repository root:  python tests/golden/make_golden.py
"""
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from castgen import configs  # noqa: E402
from oracle import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    out = {}
    p = configs.config2()
    out["config2"] = {
        "n_nodes": int(p["xyz"].shape[0]), "n_elems": int(p["conn"].shape[0]),
        "n_interface_pairs": int(p["if_a"].shape[0]),
        "dt_bound": oracle.stable_dt(p),
        "note": "128^3 jittered Kuhn tets, jitter seed 2, permutation seed 3, cast cube [0.2,0.8]^3",
    }
    del p
    c1 = configs.config1()
    out["config1"] = {"dt_bound_gershgorin": oracle.stable_dt(c1),
                      "dt_exact_bound": 2700.0 * 900.0 * (0.1 / 16) ** 2 / (2 * 150.0)}
    with open(os.path.join(HERE, "oracle_constants.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
