"""Writes fig1_points.json: full FP64 oracle solves at two settings of the
Fig. 1 phase-transition grid (Section 5.1: 100^3, Tucker rank r, R_n =
floor(1.2 r), a fraction rho corrupted by U(-1, 1), epsilon 1e-5, maxiter
1000).  Calls only the oracle and the seeded generators; run from the
repository root (about a minute per point):

    python tests/golden/make_fig1_points.py
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import pasd_solve  # noqa: E402

POINTS = [(20, 0.10, 17124600), (40, 0.10, 17124600)]


def main():
    out = {"source": "oracle/pasd_oracle.py pasd_solve, FP64", "dims": [100, 100, 100],
           "tol": 1e-5, "max_iter": 1000, "points": []}
    for r, rho, seed in POINTS:
        R = int(1.2 * r)
        wl = workloads.tucker_workload("fig1", (100, 100, 100), (r, r, r), rho, seed,
                                       ranks=(R, R, R))
        X, _, st = pasd_solve(wl.T, wl.ranks, tol=1e-5, max_iter=1000)
        rse = float(np.linalg.norm(X - wl.L) / np.linalg.norm(wl.L))
        out["points"].append({"r": r, "rho": rho, "seed": seed, "R": R, "iterations": int(st.k),
                              "rank": [int(x) for x in st.rank], "rse": rse})
        print(out["points"][-1], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "fig1_points.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
