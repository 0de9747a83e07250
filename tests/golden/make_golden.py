"""Writes tests/golden/mlp8_oracle.json from the FP64 oracle only.

The paper prints no worked numeric example, so the stored values are the
oracle's own on the 8-16-16-3 workload (seed 0), together with the exact
LP-with-cuts and MIP values of the same problem from HiGHS; the test that
reads them guards against unintended changes to the oracle.
Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import gcp_oracle as O, lp  # noqa: E402
from workloads import gen  # noqa: E402


def main():
    p = gen.make_workload("mlp8", 0)
    g, ga, gb, gc = O.bound_and_grad(p)
    out = {
        "workload": "MLP 8-16-16-3, seed 0, eps 0.05, 8 LP-implied cuts, alpha and gamma ~ U[0,1]",
        "bound": g.tolist(),
        "d_alpha": ga.tolist(),
        "d_gamma": gc.tolist(),
        "lp_cut": [lp.lp_value(p, 0, s) for s in range(p.S)],
        "mip": [lp.mip_value_enum(p, 0, s) for s in range(p.S)],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mlp8_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
