"""Write tests/golden/oracle_astar.json: homogenized coefficients computed by
the CPU oracle (and nothing else) for the full-size workloads that are too slow
to recompute inside a test.

    python tests/golden/make_golden.py            # every case
    python tests/golden/make_golden.py NAME ...   # only these; the others are kept
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2404_06841_amd import workloads as W  # noqa: E402

CASES = {
    "c2_eightfold_N16": lambda: W.eightfold(16),
    "c3_eightfold_random_N32": lambda: W.eightfold_random(32, 0),
    # diagonal coefficient diag(a_1, a_2) (App. D): the benchmark's second workload
    "diag_eightfold_N32": lambda: W.eightfold_diagonal(32, 0),
    "paper_homogenization_N18": lambda: W.paper_homogenization(18),
    # d = 3 icosahedral field at N = 10: 1,000,000 unknowns (not a power of two),
    # three correctors
    "icosa_N10": lambda: W.icosahedral(10),
    # the largest serving request and the HBM-sized product shape: d = 3,
    # n = 6, N = 16 (16,777,216 unknowns), three correctors
    "icosa_N16": lambda: W.icosahedral(16),
    # odd N = 15 (11,390,625 unknowns): the Hermitian half-storage workload
    "icosa_N15": lambda: W.icosahedral(15),
}


def main(names):
    path = os.path.join(HERE, "oracle_astar.json")
    out = {"_about": "A* (flux and energy forms) of the CPU oracle at tol 1e-12, "
                     "written by tests/golden/make_golden.py"}
    if names:
        unknown = [n for n in names if n not in CASES]
        if unknown:
            raise SystemExit(f"unknown cases {unknown}; known: {sorted(CASES)}")
        with open(path) as f:
            out.update(json.load(f))
    for name, make in CASES.items():
        if names and name not in names:
            continue
        prob = make()
        t = time.time()
        r = oracle.homogenize(prob, tol=1e-12)
        out[name] = {"N": prob.N, "D": prob.D, "tol": 1e-12,
                     "A": r.A.tolist(), "A_energy": r.A_energy.tolist(),
                     "iters": [i.iters for i in r.infos],
                     "seconds": time.time() - t}
        print(name, out[name], flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=2)


if __name__ == "__main__":
    main(sys.argv[1:])
