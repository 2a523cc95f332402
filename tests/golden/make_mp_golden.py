"""Writes mp_rounding_cases.json: two small precision-form solves by the C
oracle (``oracle.solve_mp``) with every output stored as exact hex floats.

Only the oracle and the seeded input generator are called.  Run from the
repository root: ``python tests/golden/make_mp_golden.py``.

Cases (2-D 5-point upwind convection-diffusion, 5 x 5 interior nodes,
beta = (20, 10), x_true from the seeded generator, b = A x_true, x_0 = 0):
  periodic -- tol 3e-7, replacement every 4 iterations, maxit 12;
  forced   -- tol 3e-6, no periodic replacement: the binary32 recursive
              residual passes tol before the binary64 true residual does, so
              one replacement is forced by the confirmation step.
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1612_01395_amd import inputs  # noqa: E402

CASES = {
    "periodic": dict(tol=3e-7, maxit=12, rr_period=4),
    "forced": dict(tol=3e-6, maxit=30, rr_period=0),
}


def main() -> None:
    A = oracle.assemble_workload(inputs.workload("c1", n=5))
    b = oracle.spmv(A, inputs.x_true(A.n))
    out = {
        "system": {"workload": "c1", "n": 5, "row_ptr": A.row_ptr.tolist(), "col": A.col.tolist(),
                   "val": [float(v).hex() for v in A.val], "b": [float(v).hex() for v in b]},
        "cases": {},
    }
    for name, kw in CASES.items():
        x, info = oracle.solve_mp(A, b, history=True, **kw)
        out["cases"][name] = {
            "opts": kw,
            "iters": info["iters"], "n_rr": info["n_rr"], "status": oracle.STATUS_NAMES[info["status"]],
            "x": [float(v).hex() for v in x],
            "history": [float(v).hex() for v in info["history"]],
            "relres_true": float(info["relres_true"]).hex(),
        }
    with open(os.path.join(HERE, "mp_rounding_cases.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
