"""Writes config1_oracle.json: the oracle's MatExPre solve of the 2D homogeneous
128 x 128 workload (h = 1/127, c = 1, 10 points per wavelength, 16-cell layer,
discrete delta at node (64, 64)) with t = 40 h^2, s = 1/freq, fprtol 0.08,
FGMRES(30) / inner GMRES(30) to rtol 1e-6 (Section 4 defaults; Section 3.4,
Algorithm 1).  Calls only the oracle and the seeded workload generators.

Run from the repository root:  python tests/golden/make_config1.py"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import krylov  # noqa: E402


def main():
    prob = wl.config1()
    f = wl.delta_source(prob, (64, 64)).ravel()
    t0 = time.time()
    res = krylov.matexpre_solve(prob, f, prob.default_t(), prob.default_shift(), 0.08, 1e-6,
                                outer_restart=30, inner_restart=30)
    out = {
        "workload": prob.name,
        "t": prob.default_t(),
        "shift": prob.default_shift(),
        "fprtol": 0.08,
        "rtol": 1e-6,
        "outer_iterations": res.outer_iterations,
        "inner_iterations": list(map(int, res.inner_iterations)),
        "inner_mean": res.inner_mean,
        "inner_std": res.inner_std,
        "true_relres": res.true_relres,
        "converged": bool(res.converged),
        "oracle_seconds": round(time.time() - t0, 1),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config1_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
