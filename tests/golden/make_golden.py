"""Write tests/golden/exact_opt.json: exact optimal values of small seeded
instances, computed ONLY with the oracle's exact solvers (brute force over
permutations, HiGHS LP, the monotone 1-D coupling).  No value comes from the
DROT iteration or the GPU path.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from gen import (assignment_instance, config_small_fp64, line_instance,  # noqa: E402
                 paper_protocol)
from oracle import exact  # noqa: E402


def main():
    out = {"_source": "oracle/exact.py (brute force, HiGHS, monotone coupling); "
                      "instances from gen/instances.py",
           "brute_force": [], "lp": [], "line": []}
    for n in (2, 3, 5, 7):
        for i in range(3):
            inst = assignment_instance(i, n)
            out["brute_force"].append({"n": n, "seed": i, "opt": exact.brute_force_uniform(inst.C)})
    for (m, n) in ((20, 30), (50, 50), (100, 100)):
        for i in range(2):
            inst = config_small_fp64(i, m, n)
            out["lp"].append({"gen": "config_small_fp64", "m": m, "n": n, "seed": i,
                              "opt": exact.lp_highs(inst.C, inst.p, inst.q)[0]})
    inst = paper_protocol(0, 64)
    out["lp"].append({"gen": "paper_protocol", "m": 64, "n": 64, "seed": 0,
                      "opt": exact.lp_highs(inst.C, inst.p, inst.q)[0]})
    for (m, n) in ((40, 60), (100, 80)):
        inst = line_instance(0, m, n)
        out["line"].append({"m": m, "n": n, "seed": 0,
                            "opt": exact.line_monotone(inst.xs, inst.xt, inst.C, inst.p, inst.q)[0]})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_opt.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(path)


if __name__ == "__main__":
    main()
